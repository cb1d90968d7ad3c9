"""Pins of the oracle's EM algebra (Eq. 6-9) by invariants that any correct
list-mode OS-EM iterate satisfies."""
import math

import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture(scope="module")
def tiny():
    w = synth.workload("tiny")
    act, mu = synth.phantom(w)
    g = w.geom.as_dict()
    mod = O.OracleModel(g, mu)
    ev = synth.workload_events(w, n_events=2000)
    H = mod.system_matrix(ev)
    return w, g, mod, ev, H


def test_count_conservation_and_nonnegativity(tiny):
    # after a sub-iteration sum_q sens_q^(i) f_q = number of events in subset i
    w, g, mod, ev, H = tiny
    sens = mod.sensitivity(0)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.1, 2.0, size=H.shape[1])
    f_new, mean, skipped = O.subset_update(H, f, sens)
    assert skipped == 0
    assert np.all(f_new >= 0)
    assert float(sens @ f_new) == pytest.approx(H.shape[0], rel=1e-12)
    assert np.all(mean > 0)


def test_log_likelihood_never_decreases_for_one_subset(tiny):
    w, g, mod, ev, H = tiny
    sens = mod.sensitivity(-1)[None, :]
    _f, ll = O.os_lm_mlem(H, ev["angle"], sens, 12, np.ones(H.shape[1]), 1)
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1]))


def test_update_is_degree_zero_homogeneous_and_scales_with_time(tiny):
    w, g, mod, ev, H = tiny
    sens = mod.sensitivity(0)
    f = np.linspace(0.5, 1.5, H.shape[1])
    a, _, _ = O.subset_update(H, f, sens)
    b, _, _ = O.subset_update(H, 7.5 * f, sens)
    np.testing.assert_allclose(a, b, rtol=1e-13)
    g2 = dict(g, acq_time=3.0)
    mod3 = O.OracleModel(g2, mod.mu)
    c, _, _ = O.subset_update(mod3.system_matrix(ev), f, mod3.sensitivity(0))
    np.testing.assert_allclose(c, a / 3.0, rtol=1e-12)


def test_event_order_is_irrelevant(tiny):
    w, g, mod, ev, H = tiny
    sens = mod.sensitivity(0)
    f = np.ones(H.shape[1])
    perm = np.random.default_rng(9).permutation(H.shape[0])
    a, _, _ = O.subset_update(H, f, sens)
    b, _, _ = O.subset_update(H[perm], f, sens)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_subsets_follow_angle_interleave_and_iteration_order(tiny):
    # Eq. 9: sub-iteration i starts from the estimate of sub-iteration i-1;
    # the first sub-iteration of an iteration starts from the previous
    # iteration's last one.  Subset i holds the angles a with a mod N_s == i.
    w, g, mod, ev, H = tiny
    ns = 4
    g4 = dict(g, n_subsets=ns)
    m4 = O.OracleModel(g4, mod.mu)
    sens = np.stack([m4.sensitivity(i) for i in range(ns)])
    np.testing.assert_allclose(sens.sum(axis=0), m4.sensitivity(-1), rtol=1e-12)
    f0 = np.ones(H.shape[1])
    f_os, _ = O.os_lm_mlem(H, ev["angle"], sens, 2, f0, ns)
    f = f0.copy()
    for _t in range(2):
        for i in range(ns):
            rows = ev["angle"] % ns == i
            f, _, _ = O.subset_update(H[rows], f, sens[i])
    np.testing.assert_allclose(f_os, f, rtol=1e-13)
    # one subset is plain LM-MLEM (Eq. 6)
    f1, _ = O.os_lm_mlem(H, ev["angle"], m4.sensitivity(-1)[None, :], 1, f0, 1)
    f_ref, _, _ = O.subset_update(H, f0, m4.sensitivity(-1))
    np.testing.assert_allclose(f1, f_ref, rtol=1e-14)


def test_zero_sensitivity_pixels_and_dead_events_are_handled():
    H = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 0.0]])
    f = np.array([1.0, 1.0, 3.0])
    sens = np.array([1.0, 2.0, 0.0])
    f_new, mean, skipped = O.subset_update(H, f, sens)
    assert skipped == 1                       # the third event has mean 0
    assert f_new[2] == 3.0                    # zero sensitivity: unchanged
    np.testing.assert_allclose(f_new[:2], [1.0, 0.5])


def test_binned_mlem_converges_to_the_exact_solution_of_consistent_data():
    """Consistent data y = H f_true with H of full column rank: the MLEM
    iterates converge to f_true (one subset), and with subsets every
    sub-iteration conserves its subset's counts."""
    rng = np.random.default_rng(3)
    H = rng.uniform(0.1, 1.0, size=(12, 4))
    f_true = np.array([1.0, 3.0, 0.5, 2.0])
    y = H @ f_true
    f = O.binned_os_mlem(H, y, np.zeros(12, int), 1, 4000, np.ones(4))
    np.testing.assert_allclose(f, f_true, rtol=1e-6)
    angle = np.arange(12) % 3
    f1 = O.binned_os_mlem(H, y, angle, 3, 1, np.ones(4))
    # the last sub-iteration (subset 2) conserves its counts: H_2^T 1 . f = sum y_2
    sel = angle % 3 == 2
    assert H[sel].sum(axis=0) @ f1 == pytest.approx(y[sel].sum(), rel=1e-12)
    assert np.all(f1 >= 0)


def test_binned_rows_tile_the_sensitivity():
    """Bins that tile the detector and the acceptance window integrate h over
    everything the sensitivity counts: their column sums over a subset's
    angles equal the subset sensitivity."""
    w = synth.workload("tiny")
    g = dict(w.geom.as_dict(), n_subsets=4)
    _, mu = synth.phantom(w)
    m = O.OracleModel(g, mu)
    H = O.binned_rows(m, 4, [100.0, 130.0, 175.0], angles=[1, 5, 9, 13])
    np.testing.assert_allclose(H.sum(axis=0), m.sensitivity(1), rtol=1e-10)


def test_binned_mlem_approaches_list_mode_em_as_bins_shrink():
    """Bins small enough to hold at most a few events each turn binned MLEM
    into list-mode EM: with bins that tile the detector and the window,
    sum_b H_b is the sensitivity and H_b / (H_b . f) tends to h_j / (h_j . f)
    for the event j in bin b.  On an 8x8 disk with 4 angles and 150 events the
    gap to the list-mode iterate falls as position and energy bins shrink."""
    g = synth.Geometry(8, 8, 0.8, 8, 0.8, 4, n_subsets=1)
    X, Y = synth.phantoms.pixel_centres(8, 8, 0.8)
    mu = np.where(X ** 2 + Y ** 2 <= 3.0 ** 2, 0.15, 0.0).astype(np.float32)
    act = np.where(X ** 2 + Y ** 2 <= 2.2 ** 2, 1.0, 0.0).astype(np.float32)
    act[np.hypot(X - 0.8, Y) < 0.9] = 3.0
    ev = synth.generate_events(g, act, mu, 150, 41)
    gd = g.as_dict()
    m = O.OracleModel(gd, mu)
    n_it = 3
    f_lm, _ = O.os_lm_mlem(m.system_matrix(ev), ev["angle"], m.sensitivity(-1)[None, :], n_it,
                           np.ones(len(m.support)), 1)
    gaps = []
    for n_pos, n_e in ((8, 3), (32, 12), (128, 48)):
        edges = np.linspace(gd["win_lo_kev"], gd["win_hi_kev"], n_e + 1)
        H = O.binned_rows(m, n_pos, edges)
        b = np.minimum((ev["u_bin"].astype(np.float64) * n_pos / gd["n_bins"]).astype(int), n_pos - 1)
        k = np.clip(np.searchsorted(edges, ev["energy"].astype(np.float64), side="right") - 1, 0, n_e - 1)
        y = np.bincount((ev["angle"] * n_pos + b) * n_e + k, minlength=H.shape[0]).astype(np.float64)
        np.testing.assert_allclose(H.sum(axis=0), m.sensitivity(-1), rtol=1e-9)
        f_b = O.binned_os_mlem(H, y, np.repeat(np.arange(4), n_pos * n_e), 1, n_it, np.ones(len(m.support)))
        gaps.append(float(np.max(np.abs(f_b - f_lm)) / np.max(f_lm)))
    assert gaps[0] > gaps[1] > gaps[2], gaps
    assert gaps[2] < 0.25 * gaps[0] and gaps[2] < 0.02, gaps


def test_log_likelihood_hand_values():
    """Eq. 3 without its f-independent terms, on three events and two pixels
    small enough to evaluate by hand: sum_j log(sum_q H_jq f_q) - sum_q f_q sens_q."""
    H = np.array([[1.0, 2.0], [3.0, 4.0], [0.0, 5.0]])
    f = np.array([1.0, 2.0])
    sens = np.array([4.0, 11.0])
    # means 5, 11, 10; expected count 1*4 + 2*11 = 26
    assert O.log_likelihood(H @ f, f, sens) == pytest.approx(math.log(550.0) - 26.0, rel=1e-15)


def test_os_lm_mlem_log_likelihood_and_iterate_by_hand():
    """Two subsets (angles 0, 1, 0 with N_s = 2), one iteration, evaluated by
    hand.  Subset 0 (events 0 and 2) from f = (1, 2): means 5 and 10, its
    term log 50 - f.sens0 = log 50 - 2.5, backprojection (0.2, 0.9), new
    f = (0.4, 1.8).  Subset 1 (event 1) from there: mean 8.4, term
    log 8.4 - 3.7, new f = (0.4 * (3/8.4) / 0.25, 1.8 * (4/8.4) / 2)."""
    H = np.array([[1.0, 2.0], [3.0, 4.0], [0.0, 5.0]])
    angle = np.array([0, 1, 0])
    sens = np.array([[0.5, 1.0], [0.25, 2.0]])
    f, ll = O.os_lm_mlem(H, angle, sens, 1, np.array([1.0, 2.0]), 2)
    assert ll[0] == pytest.approx(math.log(50.0) - 2.5 + math.log(8.4) - 3.7, rel=1e-14)
    np.testing.assert_allclose(f, [0.4 * (3 / 8.4) / 0.25, 1.8 * (4 / 8.4) / 2.0], rtol=1e-14)

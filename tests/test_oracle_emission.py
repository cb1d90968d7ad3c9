"""Pins of the oracle's emission set (Sec. 2.2: the estimate is confined to a
crude object boundary so that each iteration touches fewer pixels).

The boundary's growth by a disc is checked against lattice-point counts of
discs and against scipy's binary dilation; restricting the estimated pixels
is checked to be the same iteration as starting OS-LM-MLEM from an image that
is zero outside the set (multiplicative updates keep zeros)."""
import numpy as np
import pytest

import oracle as O
import synth


@pytest.mark.parametrize("margin,count", [(0, 1), (1, 5), (2, 13), (3, 29), (4, 49), (5, 81)])
def test_single_hot_pixel_grows_to_a_lattice_disc(margin, count):
    """Lattice points with i^2 + j^2 <= r^2 (Gauss circle problem)."""
    img = np.zeros((21, 21), np.float32)
    img[10, 10] = 3.0
    mu = np.full((21, 21), 0.1, np.float32)
    mask = O.emission_mask(img, mu, 0.5, margin)
    assert mask.dtype == np.float32
    assert int(mask.sum()) == count
    ii, jj = np.nonzero(mask)
    assert np.all((ii - 10) ** 2 + (jj - 10) ** 2 <= margin ** 2)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_scipy_dilation_by_a_disc(seed):
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(seed)
    img = rng.exponential(1.0, (40, 33)).astype(np.float32) * (rng.random((40, 33)) < 0.1)
    mu = (rng.random((40, 33)) < 0.8).astype(np.float32) * 0.15
    for margin in (0, 1, 2, 4):
        for t in (0.05, 0.3, 0.9):
            m = margin
            y, x = np.mgrid[-m:m + 1, -m:m + 1]
            disc = x * x + y * y <= m * m
            hot = img.astype(np.float64) >= t * float(img.max())
            ref = ndimage.binary_dilation(hot, structure=disc) & (mu > 0)
            np.testing.assert_array_equal(O.emission_mask(img, mu, t, margin) > 0, ref)


def test_zero_threshold_is_the_support_and_limits_are_monotone():
    rng = np.random.default_rng(3)
    img = rng.random((30, 30)).astype(np.float32) ** 4
    mu = (rng.random((30, 30)) < 0.7).astype(np.float32)
    np.testing.assert_array_equal(O.emission_mask(img, mu, 0.0, 0), (mu > 0).astype(np.float32))
    prev = None
    for m in range(4):
        cur = O.emission_mask(img, mu, 0.4, m)
        if prev is not None:
            assert np.all(cur >= prev)
        prev = cur
    hi, lo = O.emission_mask(img, mu, 0.6, 1), O.emission_mask(img, mu, 0.2, 1)
    assert np.all(lo >= hi)
    assert np.all(O.emission_mask(img, mu, 1.0, 0)[img < img.max()] == 0)


def test_restricted_emission_set_equals_zero_initial_estimate():
    """OS-LM-MLEM on the emission pixels only equals OS-LM-MLEM on the whole
    support started from an image that is zero off the emission set."""
    w = synth.workload("tiny")
    g = dict(w.geom.as_dict(), n_subsets=4)
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w, n_events=1500)
    m = O.OracleModel(g, mu)
    sup = m.support
    em = O.emission_mask(act, mu, 0.5, 1).ravel()[sup] > 0
    assert 0 < em.sum() < len(sup)
    H = m.system_matrix(ev)
    sens = np.stack([m.sensitivity(i) for i in range(4)])
    f_full, ll_full = O.os_lm_mlem(H, ev["angle"], sens, 5, em.astype(np.float64), 4)
    f_em, ll_em = O.os_lm_mlem(H[:, em], ev["angle"], sens[:, em], 5, np.ones(int(em.sum())), 4)
    assert np.all(f_full[~em] == 0)
    np.testing.assert_allclose(f_full[em], f_em, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(ll_full, ll_em, rtol=1e-12)
    # the restricted model's rows are the full rows' emission columns
    q_em = sup[em]
    np.testing.assert_array_equal(m.system_matrix(ev, qlist=q_em), H[:, em])

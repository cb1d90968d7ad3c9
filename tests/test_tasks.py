"""Task measures (Sec. 3: striatal uptake and its normalised RMSE over noise
realisations; image NRMSE) pinned by exact special cases and invariants."""
import numpy as np
import pytest

import synth
from paper_2002_12471_amd import tasks


@pytest.fixture(scope="module")
def brain():
    w = synth.workload("brain64")
    act, mu = synth.phantom(w)
    caud, put = synth.striatal_masks(w.geom)
    b = act > 0
    rng = np.random.default_rng(3)
    sens = np.where(mu > 0, rng.uniform(0.5, 1.5, mu.shape), 0.0)
    return dict(act=act.astype(np.float64), brain=b, caud=caud & b, put=put & b, bg=b & ~caud & ~put, sens=sens)


def test_truth_at_each_count_scale_has_zero_uptake_error(brain):
    t, s = brain["act"], brain["sens"]
    c = [0.5, 1.0, 3.0]
    counts = [k * float((s * t).sum()) for k in c]
    imgs = [k * t for k in c]
    for m in (brain["caud"], brain["put"]):
        assert tasks.uptake_nrmse(imgs, m, t, counts, s) == pytest.approx(0.0, abs=1e-14)


def test_symmetric_uptake_errors_give_their_size(brain):
    """Two realisations whose caudate is off by +eps and -eps (the rest
    exact) have caudate uptake NRMSE eps and putamen NRMSE 0."""
    t, s = brain["act"], brain["sens"]
    counts = [float((s * t).sum())] * 2
    eps = 0.125
    up, down = t.copy(), t.copy()
    up[brain["caud"]] *= 1 + eps
    down[brain["caud"]] *= 1 - eps
    assert tasks.uptake_nrmse([up, down], brain["caud"], t, counts, s) == pytest.approx(eps, rel=1e-12)
    assert tasks.uptake_nrmse([up, down], brain["put"], t, counts, s) == pytest.approx(0.0, abs=1e-14)


def test_phantom_ratios_are_eight_and_scale_free(brain):
    t = brain["act"]
    for m in (brain["caud"], brain["put"]):
        r = tasks.region_ratios([t, 2.5 * t], m, brain["bg"])
        np.testing.assert_allclose(r, [8.0, 8.0], rtol=1e-14)


def test_image_nrmse_special_cases(brain):
    """Zero for the truth at any scale; for an image constant over the brain
    it is the truth's coefficient of variation over its root mean square,
    sqrt(var / mean of squares), from the counts of the two phantom values."""
    t, b = brain["act"], brain["brain"]
    np.testing.assert_allclose(tasks.image_nrmse([t, 7.0 * t], t, b), [0.0, 0.0], atol=1e-14)
    n = int(b.sum())
    n8 = int((t[b] == 8.0).sum())
    assert n8 > 0 and int((t[b] == 1.0).sum()) == n - n8
    mean = (n8 * 8.0 + (n - n8) * 1.0) / n
    meansq = (n8 * 64.0 + (n - n8) * 1.0) / n
    flat = np.where(b, 0.3, 0.0)
    got = tasks.image_nrmse([flat], t, b)[0]
    assert got == pytest.approx(np.sqrt((meansq - mean ** 2) / meansq), rel=1e-12)


def test_empty_regions_are_rejected(brain):
    t, s = brain["act"], brain["sens"]
    none = np.zeros_like(brain["brain"])
    with pytest.raises(ValueError):
        tasks.uptake_nrmse([t], none, t, [1.0], s)
    with pytest.raises(ValueError):
        tasks.region_ratios([t], brain["caud"], none)
    with pytest.raises(ValueError):
        tasks.image_nrmse([t], t, none)

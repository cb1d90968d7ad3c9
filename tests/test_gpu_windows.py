"""GPU parity for the acceptance windows of the paper's experiment matrix
(Sec. 3: photopeak only, 143-175 keV, and 120-175 keV, beside the whole
100-175 keV spectrum that the other tests use): the same events restricted to
each window, reconstructed by a context whose window is that range, against
the FP64 oracle with the same window.

Tolerances as in test_gpu_parity: per event |g - o| <= 1e-4 o; per pixel
|g - o| <= 1e-3 o where o >= 1e-2 max(o), else <= 1e-5 max(o); sensitivity
<= 2e-6 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
import synth  # noqa: E402

WINDOWS = [(143.0, 175.0), (120.0, 175.0)]


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


def _rel(g, o):
    return np.abs(np.asarray(g, np.float64) - o) / np.abs(o)


def _image_ok(got, ref):
    err = np.abs(np.asarray(got, np.float64) - ref)
    tol = np.where(ref >= 1e-2 * ref.max(), 1e-3 * ref, 1e-5 * ref.max())
    return bool(np.all(err <= tol)), float(np.max(err / np.maximum(np.abs(ref), 1e-300)))


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _in_window(ev, lo, hi):
    sel = (ev["energy"] >= lo) & (ev["energy"] <= hi)
    return {k: ev[k][sel] for k in ("angle", "u_bin", "energy")}


@pytest.mark.parametrize("lo,hi", WINDOWS)
def test_window_tiny_sensitivity_means_and_10_iterations(dev, lo, hi):
    L = _lib()
    w = synth.workload("tiny")
    act, mu = synth.phantom(w)
    g = dict(w.geom.as_dict(), win_lo_kev=lo, win_hi_kev=hi)
    ev = _in_window(synth.workload_events(w), lo, hi)
    print(f"window [{lo}, {hi}] keV: {len(ev['angle'])} of {w.n_events} events", flush=True)
    assert 0.5 * w.n_events < len(ev["angle"]) < w.n_events
    m = O.OracleModel(g, mu)
    H = m.system_matrix(ev)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        sens = ctx.sensitivity(-1).cpu().numpy().ravel()[m.support]
        assert np.max(_rel(sens, m.sensitivity(-1))) <= 2e-6
        evd = L.events_to_device(ev, dev)
        got = ctx.forward(evd, torch.as_tensor(act, device=dev)).cpu().numpy()
        ref = H @ act.ravel()[m.support].astype(np.float64)
        assert np.max(_rel(got, ref)) <= 1e-4
        img, ll = ctx.reconstruct(evd, 10, want_loglik=True)
    finally:
        ctx.close()
    f_ref, ll_ref = O.os_lm_mlem(H, ev["angle"], m.sensitivity(-1)[None, :], 10, np.ones(len(m.support)), 1)
    ok, worst = _image_ok(img.cpu().numpy().ravel()[m.support], f_ref)
    assert ok, worst
    np.testing.assert_allclose(ll[0], ll_ref, rtol=1e-5)


@pytest.mark.parametrize("lo,hi", WINDOWS)
def test_window_brain64_sampled_means_and_subset_update(dev, lo, hi):
    """brain64 with the window's events: every event of the window in one
    forward launch (the oracle computes 128 sampled events), then one
    sub-iteration of subset 2 against the oracle's update."""
    L = _lib()
    w = synth.workload("brain64")
    act, mu = synth.phantom(w)
    g = dict(w.geom.as_dict(), win_lo_kev=lo, win_hi_kev=hi)
    ev = _in_window(synth.workload_events(w, realisation=3, n_events=40_000), lo, hi)
    m = O.OracleModel(g, mu)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        evd = L.events_to_device(ev, dev)
        got = ctx.forward(evd, torch.as_tensor(act, device=dev)).cpu().numpy()
        idx = np.sort(np.random.default_rng(7).choice(len(got), 128, replace=False))
        ref = m.system_matrix({k: v[idx] for k, v in ev.items()}) @ act.ravel()[m.support].astype(np.float64)
        assert np.max(_rel(got[idx], ref)) <= 1e-4
        sel = ev["angle"] % g["n_subsets"] == 2
        sub = {k: v[sel][:1500] for k, v in ev.items()}
        img = torch.as_tensor((mu > 0).astype(np.float32), device=dev)
        ctx.subset_update(2, L.events_to_device(sub, dev), img)
        got_img = img.cpu().numpy().ravel()[m.support]
    finally:
        ctx.close()
    f_ref, _, skipped = O.subset_update(m.system_matrix(sub), np.ones(len(m.support)), m.sensitivity(2))
    assert skipped == 0
    ok, worst = _image_ok(got_img, f_ref)
    assert ok, worst

"""GPU tests of cached system rows: the rows h_j(q) do not depend on the
estimate, so a prepared set may keep them after the first iteration and read
them back in every later sub-iteration.  Checked against the FP64 oracle and
against the recomputing path (which differs only in FP32 summation order)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
import synth  # noqa: E402


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _image_ok(got, ref):
    err = np.abs(np.asarray(got, np.float64) - ref)
    tol = np.where(ref >= 1e-2 * ref.max(), 1e-3 * ref, 1e-5 * ref.max())
    return np.all(err <= tol), float(np.max(err / np.maximum(np.abs(ref), 1e-300)))


def _iterate(L, ctx, evd, mu, n_iters, cache, offsets=None, calls=1, tune=False, want_ll=False):
    """n_iters iterations on a prepared set, split over `calls` calls."""
    R = 1 if offsets is None else len(offsets) - 1
    evs = L.lmosem_events_load(ctx.handle, evd, offsets)
    try:
        if tune:
            L.lmosem_autotune(ctx.handle, evs)
        if cache:
            L.lmosem_cache_rows(ctx.handle, evs, True)
        img = torch.as_tensor(np.broadcast_to((mu > 0).astype(np.float32), (R,) + mu.shape).copy(),
                              device=evd["angle"].device)
        lls = []
        per = n_iters // calls
        for _ in range(calls):
            ll = L.lmosem_iterate(ctx.handle, evs, per, img, n_real=R, want_loglik=want_ll)
            if want_ll:
                lls.append(ll)
        torch.cuda.synchronize()
        return img.cpu().numpy(), (np.concatenate(lls, axis=1) if want_ll else None)
    finally:
        L.lmosem_events_free(evs)


def test_cached_rows_tiny_10_iterations_match_oracle(dev):
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        img, ll = _iterate(L, ctx, L.events_to_device(ev, dev), mu, 10, cache=True, want_ll=True)
    finally:
        ctx.close()
    m = O.OracleModel(g, mu)
    f_ref, ll_ref = O.os_lm_mlem(m.system_matrix(ev), ev["angle"], m.sensitivity(-1)[None, :], 10,
                                 np.ones(len(m.support)), 1)
    ok, worst = _image_ok(img[0].ravel()[m.support], f_ref)
    assert ok, worst
    np.testing.assert_allclose(ll[0], ll_ref, rtol=1e-5)


def test_cached_rows_brain64_equal_recomputed(dev):
    """Full brain64 set (200k events, 8 subsets), autotuned, graphs as tuned:
    4 iterations over two calls with cached rows (the second call replays the
    cached-row graph) against 4 recomputing iterations."""
    L = _lib()
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    evd = L.events_to_device(synth.workload_events(w), dev)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        ref, ll_ref = _iterate(L, ctx, evd, mu, 4, cache=False, tune=True, want_ll=True)
        got, ll = _iterate(L, ctx, evd, mu, 4, cache=True, calls=2, tune=True, want_ll=True)
    finally:
        ctx.close()
    sup = mu.ravel() > 0
    r, gg = ref[0].ravel()[sup].astype(np.float64), got[0].ravel()[sup]
    assert np.max(np.abs(gg - r) / np.maximum(r, 1e-3 * r.max())) <= 1e-4
    np.testing.assert_allclose(ll, ll_ref, rtol=1e-6)


def test_cached_rows_batched_realisations(dev):
    """Three realisations of uneven size in one set, with the cache enabled
    after autotuning, against the recomputing path."""
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    parts = [synth.workload_events(w, realisation=r, n_events=n) for r, n in enumerate((3000, 700, 5000))]
    ev = {k: np.concatenate([p[k] for p in parts]) for k in ("angle", "u_bin", "energy")}
    offsets = [0, 3000, 3700, 8700]
    ctx = L.Context(dict(g, n_subsets=4), torch.as_tensor(mu, device=dev))
    try:
        evd = L.events_to_device(ev, dev)
        ref, _ = _iterate(L, ctx, evd, mu, 5, cache=False, offsets=offsets)
        got, _ = _iterate(L, ctx, evd, mu, 5, cache=True, offsets=offsets, calls=5, tune=True)
    finally:
        ctx.close()
    sup = mu.ravel() > 0
    for r in range(3):
        a, b = ref[r].ravel()[sup].astype(np.float64), got[r].ravel()[sup]
        assert np.max(np.abs(b - a) / np.maximum(a, 1e-3 * a.max())) <= 1e-4, r


def test_cached_rows_many_realisations(dev):
    """More realisations (1100, two of them empty) than the row kernel keeps
    offsets for in LDS, so it looks each row's realisation up in memory:
    cached rows against the recomputing path."""
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    sizes = np.random.default_rng(5).integers(1, 40, size=1100)
    sizes[[3, 500]] = 0
    ev = synth.workload_events(w, n_events=int(sizes.sum()))
    offsets = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    ctx = L.Context(dict(g, n_subsets=4), torch.as_tensor(mu, device=dev))
    try:
        evd = L.events_to_device(ev, dev)
        ref, _ = _iterate(L, ctx, evd, mu, 3, cache=False, offsets=offsets)
        got, _ = _iterate(L, ctx, evd, mu, 3, cache=True, offsets=offsets, calls=3)
    finally:
        ctx.close()
    sup = mu.ravel() > 0
    a, b = ref.reshape(len(sizes), -1)[:, sup].astype(np.float64), got.reshape(len(sizes), -1)[:, sup]
    assert np.all(np.isfinite(b))
    assert np.max(np.abs(b - a) / np.maximum(a, 1e-3 * a.max())) <= 1e-4


def test_cached_rows_learned_scatter(dev):
    """A learned-scatter context: rows from the network's path, cached after
    the first iteration, against recomputing them every iteration."""
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    p = synth.mlp_init_params(3)   # an untrained network: any output is a valid test of caching
    net = L.lmosem_net_create(p)
    ctx = L.Context(dict(g, scatter_model=2), torch.as_tensor(mu, device=dev))
    try:
        L.lmosem_set_surrogate(ctx.handle, net)
        evd = L.events_to_device(synth.workload_events(w), dev)
        ref, _ = _iterate(L, ctx, evd, mu, 3, cache=False)
        got, _ = _iterate(L, ctx, evd, mu, 3, cache=True, calls=3)
    finally:
        ctx.close()
        L.lmosem_net_destroy(net)
    sup = mu.ravel() > 0
    a, b = ref[0].ravel()[sup].astype(np.float64), got[0].ravel()[sup]
    assert np.max(np.abs(b - a) / np.maximum(a, 1e-3 * a.max())) <= 1e-4


def test_cached_rows_large_support(dev):
    """A support of 17k pixels (150x150 disk of radius 74 px, 8 angles, rows
    of 69 KB) with cached rows against the recomputing path."""
    L = _lib()
    g = synth.Geometry(150, 150, 0.1, 160, 0.1, 8, n_subsets=2)
    X, Y = synth.phantoms.pixel_centres(150, 150, 0.1)
    mu = np.where(X ** 2 + Y ** 2 <= (74 * 0.1) ** 2, 0.15, 0.0).astype(np.float32)
    act = np.where(X ** 2 + Y ** 2 <= (60 * 0.1) ** 2, 1.0, 0.0).astype(np.float32)
    assert int((mu > 0).sum()) > 16384
    ev = synth.generate_events(g, act, mu, 3000, 77)
    ctx = L.Context(g.as_dict(), torch.as_tensor(mu, device=dev))
    try:
        evd = L.events_to_device(ev, dev)
        ref, _ = _iterate(L, ctx, evd, mu, 3, cache=False)
        got, _ = _iterate(L, ctx, evd, mu, 3, cache=True, calls=3)
    finally:
        ctx.close()
    sup = mu.ravel() > 0
    a, b = ref[0].ravel()[sup].astype(np.float64), got[0].ravel()[sup]
    assert np.max(np.abs(b - a) / np.maximum(a, 1e-3 * a.max())) <= 1e-4

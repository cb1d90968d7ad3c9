"""GPU parity at the full workload sizes, in the launch configuration the
bench times (prepared event sets, autotuned event tiles and chunks): sampled
outputs that the FP64 oracle computes one by one, and invariants that hold at
any size.

Tolerances as in test_gpu_parity: per event |g - o| <= 1e-4 o; per pixel
|g - o| <= 1e-3 o where o >= 1e-2 max(o), else <= 1e-5 max(o).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
import synth  # noqa: E402


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


def _rel(g, o):
    return np.abs(np.asarray(g, np.float64) - o) / np.abs(o)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def test_brain128_subset_forward_sampled_events(dev):
    """The 128x128 brain: all events of subset 0 of the 2M (one forward launch
    of the bench's sub-iteration, ~133k events) with the event tile the
    autotuner picks for the whole set; the oracle computes 48 sampled events."""
    L = _lib()
    w = synth.workload("brain128")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        evs = L.lmosem_events_load(ctx.handle, L.events_to_device(ev, dev))
        tile, _, _ = L.lmosem_autotune(ctx.handle, evs)
        L.lmosem_events_free(evs)
        print(f"autotuned event tile {tile}")
        ctx.set_tuning(tile)
        sel = np.flatnonzero(ev["angle"] % g["n_subsets"] == 0)
        sub = {k: ev[k][sel] for k in ("angle", "u_bin", "energy")}
        got = ctx.forward(L.events_to_device(sub, dev), torch.as_tensor(act, device=dev)).cpu().numpy()
    finally:
        ctx.close()
    m = O.OracleModel(g, mu)
    idx = np.sort(np.random.default_rng(12).choice(len(sel), 48, replace=False))
    ref = m.system_matrix({k: v[idx] for k, v in sub.items()}) @ act.ravel()[m.support].astype(np.float64)
    live = ref > 0
    assert live.sum() >= 40
    assert np.max(_rel(got[idx][live], ref[live])) <= 1e-4
    assert np.all(got[idx][~live] == 0)


def test_batch_tiny_all_realisations_one_iteration(dev):
    """All 64 realisations of uneven size (13.8M events) through one autotuned
    iteration of the prepared-set path: in every realisation the update
    conserves the events that have a positive mean (sens . f = J_r - dead_r),
    and the smallest realisation matches the oracle's update."""
    L = _lib()
    w = synth.workload("batch_tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    sizes = synth.batch_event_counts(w)
    parts = [synth.workload_events(w, realisation=r, n_events=int(n)) for r, n in enumerate(sizes)]
    ev = {k: np.concatenate([p[k] for p in parts]) for k in ("angle", "u_bin", "energy")}
    offsets = [0] + list(np.cumsum(sizes).astype(int))
    R = len(sizes)
    start = (mu > 0).astype(np.float32)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        evd = L.events_to_device(ev, dev)
        # events with zero mean at the start image are skipped in the first iteration
        m0 = ctx.forward(evd, torch.as_tensor(start, device=dev)).cpu().numpy()
        evs = L.lmosem_events_load(ctx.handle, evd, offsets)
        tile, chunk, graphs = L.lmosem_autotune(ctx.handle, evs)
        print(f"autotuned: tile {tile}, chunk {chunk}, graphs {graphs}")
        img = torch.as_tensor(np.broadcast_to(start, (R,) + mu.shape).copy(), device=dev)
        L.lmosem_iterate(ctx.handle, evs, 1, img, n_real=R)
        L.lmosem_events_free(evs)
        sens = ctx.sensitivity(0).double()
        imgs = img.double()
        for r in range(R):
            live = int((m0[offsets[r]:offsets[r + 1]] > 0).sum())
            assert float((sens * imgs[r]).sum()) == pytest.approx(live, rel=1e-5), r
        got = img.cpu().numpy()
    finally:
        ctx.close()
    r0 = int(np.argmin(sizes))
    m = O.OracleModel(g, mu)
    H = m.system_matrix(parts[r0])
    sens_o = np.stack([m.sensitivity(0)])
    f_ref, _ = O.os_lm_mlem(H, parts[r0]["angle"], sens_o, 1, np.ones(len(m.support)), 1)
    gr = got[r0].ravel()[m.support].astype(np.float64)
    err = np.abs(gr - f_ref)
    tol = np.where(f_ref >= 1e-2 * f_ref.max(), 1e-3 * f_ref, 1e-5 * f_ref.max())
    assert np.all(err <= tol), float(np.max(err / np.maximum(f_ref, 1e-300)))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """Stored oracle results (tests/golden/make_golden.py: FP64 oracle on the
    seeded synthetic inputs; nothing in them comes from the GPU library)."""
    path = os.path.join(GOLDEN, name)
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _checksums(ev):
    return np.array([len(ev["angle"]), float(np.sum(ev["angle"].astype(np.int64))),
                     float(np.sum(ev["u_bin"].astype(np.float64))), float(np.sum(ev["energy"].astype(np.float64)))])


def test_brain64_full_size_10_iterations_match_oracle(dev):
    """The 64x64 brain at full size in the bench's launch configuration: all
    200,000 events of realisation 0 as one prepared set (8 subsets of about
    25k events, so each update adds about 100-200 backprojection chunk
    partials), autotuned, one lmosem_iterate call per global iteration; the
    estimate after each of the 10 iterations against the oracle's OS-LM-MLEM
    (Eq. 7-9) on the same events, per pixel, and the per-iteration sum of
    the subsets' Eq. 3 terms from a second, lmosem_reconstruct run."""
    L = _lib()
    gold = _golden("brain64_full_os.npz")
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    np.testing.assert_array_equal(_checksums(ev), gold["event_checksums"],
                                  err_msg="the event generator no longer reproduces the stored oracle's inputs")
    sup = gold["support"]
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        for subset in (0, 7):
            s = ctx.sensitivity(subset).cpu().numpy().ravel()[sup]
            assert np.max(_rel(s, gold["sens"][subset])) <= 2e-6
        evd = L.events_to_device(ev, dev)
        evs = L.lmosem_events_load(ctx.handle, evd)
        tile, chunk, graphs = L.lmosem_autotune(ctx.handle, evs)
        print(f"autotuned: tile {tile}, chunk {chunk}, graphs {graphs}", flush=True)
        img = torch.as_tensor((mu > 0).astype(np.float32), device=dev).contiguous()
        worst = []
        for it in range(10):
            L.lmosem_iterate(ctx.handle, evs, 1, img)
            got = img.cpu().numpy().ravel()[sup]
            ref = gold["images"][it]
            err = np.abs(got.astype(np.float64) - ref)
            tol = np.where(ref >= 1e-2 * ref.max(), 1e-3 * ref, 1e-5 * ref.max())
            worst.append(float(np.max(err / tol)))
            assert np.all(err <= tol), (it, worst[-1])
        L.lmosem_events_free(evs)
        print("worst error / tolerance per iteration:", " ".join(f"{x:.3f}" for x in worst), flush=True)
        img2, ll = ctx.reconstruct(evd, 10, want_loglik=True)
        np.testing.assert_allclose(ll[0], gold["loglik"], rtol=1e-5)
        np.testing.assert_allclose(img2.cpu().numpy().ravel()[sup], img.cpu().numpy().ravel()[sup],
                                   rtol=1e-5, atol=1e-7 * float(img.max()))
    finally:
        ctx.close()


def test_brain128_exact_means_on_the_oracle_subsample(dev):
    """The 128x128 brain: per-event means at the true activity for the seeded
    64k-event subsample of the 2M events, in one forward launch with the event
    tile the autotuner picks for the whole set, against the stored FP64
    oracle means: |g - o| <= 1e-4 o for every event the oracle gives a
    positive mean, and exactly 0 for the others."""
    L = _lib()
    gold = _golden("brain128_means.npz")
    w = synth.workload("brain128")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    np.testing.assert_array_equal(_checksums(ev), gold["event_checksums"],
                                  err_msg="the event generator no longer reproduces the stored oracle's inputs")
    idx = gold["index"]
    sub = {k: ev[k][idx] for k in ("angle", "u_bin", "energy")}
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        evs = L.lmosem_events_load(ctx.handle, L.events_to_device(ev, dev))
        tile, _, _ = L.lmosem_autotune(ctx.handle, evs)
        L.lmosem_events_free(evs)
        ctx.set_tuning(tile)
        got = ctx.forward(L.events_to_device(sub, dev), torch.as_tensor(act, device=dev)).cpu().numpy()
    finally:
        ctx.close()
    ref = gold["means"]
    live = ref > 0
    print(f"{live.sum()} of {len(ref)} events with a positive mean; tile {tile}; "
          f"max rel err {np.max(_rel(got[live], ref[live])):.2e}", flush=True)
    assert live.sum() >= 0.99 * len(ref)
    assert np.max(_rel(got[live], ref[live])) <= 1e-4
    assert np.all(got[~live] == 0)

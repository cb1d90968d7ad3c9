"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Tolerances (FP32 path against FP64 oracle):
  per-event mean   |g - o| <= 1e-4 o for every event
  per-pixel image  |g - o| <= 1e-3 o where o >= 1e-2 max(o), else <= 1e-5 max(o)
  sensitivity      |g - o| <= 2e-6 o   (FP64 sums rounded once to FP32)
"""
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


def _image_ok(got, ref):
    err = np.abs(np.asarray(got, np.float64) - ref)
    tol = np.where(ref >= 1e-2 * ref.max(), 1e-3 * ref, 1e-5 * ref.max())
    return np.all(err <= tol), float(np.max(err / np.maximum(np.abs(ref), 1e-300)))


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def tiny(dev):
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    m = O.OracleModel(g, mu)
    H = m.system_matrix(ev)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    return dict(L=L, w=w, g=g, act=act, mu=mu, ev=ev, m=m, H=H, ctx=ctx,
                evd=L.events_to_device(ev, dev))


def test_sensitivity_matches_oracle(tiny):
    m, ctx = tiny["m"], tiny["ctx"]
    for subset in (-1, 0):
        got = ctx.sensitivity(subset).cpu().numpy().ravel()[m.support]
        ref = m.sensitivity(subset)
        assert np.max(_rel(got, ref)) <= 2e-6
    # zero off the support
    img = ctx.sensitivity(-1).cpu().numpy().ravel()
    off = np.setdiff1d(np.arange(img.size), m.support)
    assert np.all(img[off] == 0)


@pytest.mark.parametrize("which", ["truth", "ones"])
def test_forward_means_tiny(tiny, dev, which):
    m, ctx, H = tiny["m"], tiny["ctx"], tiny["H"]
    img = tiny["act"] if which == "truth" else (tiny["mu"] > 0).astype(np.float32)
    got = ctx.forward(tiny["evd"], torch.as_tensor(img, device=dev)).cpu().numpy()
    ref = H @ img.ravel()[m.support].astype(np.float64)
    assert np.max(_rel(got, ref)) <= 1e-4


@pytest.mark.parametrize("tile,pixels", [(8, 0), (16, 0), (32, 0), (8, 64), (32, 64), (16, 128), (8, 256)])
def test_event_tile_sizes_agree(tiny, dev, tile, pixels):
    # event tiles x pixel tiles (0: the default, the 192-pixel emission set in
    # one workgroup; 256 leaves one wave of each workgroup idle)
    m, ctx, H = tiny["m"], tiny["ctx"], tiny["H"]
    ctx.set_tuning(tile, pixels)
    try:
        img = torch.as_tensor(tiny["act"], device=dev)
        got = ctx.forward(tiny["evd"], img).cpu().numpy()
    finally:
        ctx.set_tuning(0)
    ref = H @ tiny["act"].ravel()[m.support].astype(np.float64)
    assert np.max(_rel(got, ref)) <= 1e-4


def test_backprojection_tiny(tiny, dev):
    m, ctx, H = tiny["m"], tiny["ctx"], tiny["H"]
    w = synth.random_weights(len(tiny["ev"]["angle"]), 77)
    got = ctx.backproject(tiny["evd"], torch.as_tensor(w, device=dev)).cpu().numpy().ravel()[m.support]
    ref = H.T @ w.astype(np.float64)
    assert np.max(_rel(got, ref)) <= 1e-4


def test_subset_update_tiny(tiny, dev):
    m, ctx, H = tiny["m"], tiny["ctx"], tiny["H"]
    img = torch.as_tensor((tiny["mu"] > 0).astype(np.float32), device=dev)
    mean = ctx.subset_update(0, tiny["evd"], img)
    f_ref, mean_ref, skipped = O.subset_update(H, np.ones(len(m.support)), m.sensitivity(0))
    assert skipped == 0
    assert np.max(_rel(mean.cpu().numpy(), mean_ref)) <= 1e-4
    ok, worst = _image_ok(img.cpu().numpy().ravel()[m.support], f_ref)
    assert ok, worst
    # count conservation: sum_q sens_q f_q = number of events
    sens = ctx.sensitivity(0).double()
    assert float((sens * img.double()).sum()) == pytest.approx(len(mean_ref), rel=1e-5)


def test_reconstruct_tiny_10_iterations(tiny, dev):
    m, ctx, H = tiny["m"], tiny["ctx"], tiny["H"]
    img, ll = ctx.reconstruct(tiny["evd"], 10, want_loglik=True)
    sens = m.sensitivity(-1)[None, :]
    f_ref, ll_ref = O.os_lm_mlem(H, tiny["ev"]["angle"], sens, 10, np.ones(len(m.support)), 1)
    ok, worst = _image_ok(img.cpu().numpy().ravel()[m.support], f_ref)
    assert ok, worst
    assert np.allclose(ll[0], ll_ref, rtol=1e-5)
    assert np.all(np.diff(ll[0]) >= -1e-6 * np.abs(ll[0][:-1]))


def test_reconstruct_is_deterministic(tiny):
    ctx = tiny["ctx"]
    a = ctx.reconstruct(tiny["evd"], 3).cpu().numpy()
    b = ctx.reconstruct(tiny["evd"], 3).cpu().numpy()
    assert np.array_equal(a, b)


def test_batched_realisations_equal_single_runs(tiny, dev):
    L, g, mu = tiny["L"], tiny["g"], tiny["mu"]
    w = tiny["w"]
    sizes = [1500, 37, 0, 2600]
    evs = [synth.workload_events(w, realisation=10 + k, n_events=n) if n else
           {"angle": np.zeros(0, np.int32), "u_bin": np.zeros(0, np.float32),
            "energy": np.zeros(0, np.float32)} for k, n in enumerate(sizes)]
    g2 = dict(g, n_subsets=4)
    ctx = L.Context(g2, torch.as_tensor(mu, device=dev))
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("angle", "u_bin", "energy")}
    offs = np.concatenate([[0], np.cumsum(sizes)])
    batch = ctx.reconstruct(L.events_to_device(cat, dev), 3, batch_offsets=list(offs)).cpu().numpy()
    for k, e in enumerate(evs):
        single = ctx.reconstruct(L.events_to_device(e, dev), 3).cpu().numpy()
        assert np.array_equal(batch[k], single), k
    ctx.close()


def test_empty_event_list_gives_zero_image(tiny, dev):
    L, ctx, m = tiny["L"], tiny["ctx"], tiny["m"]
    empty = {"angle": torch.zeros(0, dtype=torch.int32, device=dev),
             "u_bin": torch.zeros(0, dtype=torch.float32, device=dev),
             "energy": torch.zeros(0, dtype=torch.float32, device=dev)}
    img = ctx.reconstruct(empty, 2).cpu().numpy()
    assert np.all(img == 0)


def test_invalid_inputs_are_rejected(tiny, dev):
    L, ctx = tiny["L"], tiny["ctx"]
    ev = {k: v.clone() for k, v in tiny["evd"].items()}
    ev["angle"][3] = 99
    ev["energy"][5] = 400.0
    with pytest.raises(L.LmosemError) as ei:
        ctx.reconstruct(ev, 1)
    assert ei.value.status == L.ERANGE
    assert "2 events" in str(ei.value)
    bad_mu = torch.full((16, 16), -1.0, device=dev)
    with pytest.raises(L.LmosemError):
        L.Context(tiny["g"], bad_mu)
    with pytest.raises(L.LmosemError):
        L.Context(dict(tiny["g"], n_subsets=0), torch.as_tensor(tiny["mu"], device=dev))
    # the context stays usable after ERANGE
    assert ctx.reconstruct(tiny["evd"], 1).abs().sum().item() > 0


@pytest.fixture(scope="module")
def brain(dev):
    L = _lib()
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    m = O.OracleModel(g, mu)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    return dict(L=L, w=w, g=g, act=act, mu=mu, ev=ev, m=m, ctx=ctx, evd=L.events_to_device(ev, dev))


@pytest.fixture(scope="module")
def brain_sparse(brain):
    # about three events per angle: a tile's events spread over the whole
    # detector, so its path ends take many staging passes of 128 ranks
    m, w = brain["m"], brain["w"]
    ev = synth.workload_events(w, realisation=9, n_events=400)
    ref = m.system_matrix(ev) @ brain["act"].ravel()[m.support].astype(np.float64)
    return dict(ev=ev, ref=ref)


@pytest.mark.parametrize("tile,pixels", [(8, 64), (16, 64), (32, 64), (8, 256), (16, 256), (32, 256)])
def test_brain_sparse_tiles_match_oracle(brain, brain_sparse, dev, tile, pixels):
    L, ctx = brain["L"], brain["ctx"]
    ctx.set_tuning(tile, pixels)
    try:
        got = ctx.forward(L.events_to_device(brain_sparse["ev"], dev),
                          torch.as_tensor(brain["act"], device=dev)).cpu().numpy()
    finally:
        ctx.set_tuning(0)
    ref = brain_sparse["ref"]
    live = ref > 0
    assert live.sum() >= 0.95 * len(ref)
    assert np.max(_rel(got[live], ref[live])) <= 1e-4 and np.all(got[~live] == 0)


def test_sensitivity_brain(brain):
    m, ctx = brain["m"], brain["ctx"]
    for subset in (0, 5):
        got = ctx.sensitivity(subset).cpu().numpy().ravel()[m.support]
        assert np.max(_rel(got, m.sensitivity(subset))) <= 2e-6


def test_forward_full_size_sampled_events(brain, dev):
    # all 200k events in one launch; the oracle computes 192 of them
    m, ctx, ev = brain["m"], brain["ctx"], brain["ev"]
    img = brain["act"]
    got = ctx.forward(brain["evd"], torch.as_tensor(img, device=dev)).cpu().numpy()
    idx = np.sort(np.random.default_rng(2).choice(len(got), 192, replace=False))
    sub = {k: ev[k][idx] for k in ("angle", "u_bin", "energy")}
    ref = m.system_matrix(sub) @ img.ravel()[m.support].astype(np.float64)
    assert np.max(_rel(got[idx], ref)) <= 1e-4


def test_backprojection_full_subset_sampled_pixels(brain, dev):
    m, ctx, ev = brain["m"], brain["ctx"], brain["ev"]
    sel = ev["angle"] % brain["g"]["n_subsets"] == 3
    sub = {k: ev[k][sel] for k in ("angle", "u_bin", "energy")}
    w = synth.random_weights(int(sel.sum()), 5)
    got = ctx.backproject(brain["L"].events_to_device(sub, dev), torch.as_tensor(w, device=dev))
    got = got.cpu().numpy().ravel()
    q = np.sort(np.random.default_rng(4).choice(m.support, 12, replace=False)).astype(np.int32)
    ref = m.system_matrix(sub, q).T @ w.astype(np.float64)
    assert np.max(_rel(got[q], ref)) <= 1e-4


def test_full_size_iteration_conserves_counts(brain, dev):
    L, ctx, g = brain["L"], brain["ctx"], brain["g"]
    evs = L.lmosem_events_load(ctx.handle, brain["evd"])
    try:
        img = torch.as_tensor((brain["mu"] > 0).astype(np.float32), device=dev).contiguous()
        L.lmosem_iterate(ctx.handle, evs, 1, img)
        # after the last sub-iteration of subset N_s-1, sens^(N_s-1) . f = J_(N_s-1)
        last = g["n_subsets"] - 1
        j_last = int((brain["ev"]["angle"] % g["n_subsets"] == last).sum())
        s = ctx.sensitivity(last).double()
        assert float((s * img.double()).sum()) == pytest.approx(j_last, rel=1e-5)
        assert float(img.min()) >= 0
    finally:
        L.lmosem_events_free(evs)


def test_reconstruct_brain_geometry_small_event_count(brain, dev):
    # 2000 events over 8 subsets x 10 iterations: small enough for the oracle
    m, ctx, w = brain["m"], brain["ctx"], brain["w"]
    ev = synth.workload_events(w, realisation=5, n_events=2000)
    img = ctx.reconstruct(brain["L"].events_to_device(ev, dev), 10).cpu().numpy()
    H = m.system_matrix(ev)
    ns = brain["g"]["n_subsets"]
    sens = np.stack([m.sensitivity(i) for i in range(ns)])
    f_ref, _ = O.os_lm_mlem(H, ev["angle"], sens, 10, np.ones(len(m.support)), ns)
    ok, worst = _image_ok(img.ravel()[m.support], f_ref)
    assert ok, worst


def test_graph_replays_match_kernel_by_kernel(tiny, dev):
    # every replay of the captured iteration is compared with the same
    # iteration launched kernel by kernel, with eager work in between
    L, ctx, mu = tiny["L"], tiny["ctx"], tiny["mu"]
    g4 = dict(tiny["g"], n_subsets=4)
    c4 = L.Context(g4, torch.as_tensor(mu, device=dev))
    ev = L.lmosem_events_load(c4.handle, tiny["evd"])
    try:
        start = torch.as_tensor((mu > 0).astype(np.float32), device=dev)
        a = start.clone()
        b = start.clone()
        for it in range(4):
            want_ll = it % 2 == 1
            L.lmosem_set_graphs(c4.handle, False)
            ll_a = L.lmosem_iterate(c4.handle, ev, 1, a, want_loglik=want_ll)
            junk = torch.randn(4096, device=dev).cumsum(0)   # unrelated eager work
            torch.cuda.synchronize()
            L.lmosem_set_graphs(c4.handle, True)
            ll_b = L.lmosem_iterate(c4.handle, ev, 1, b, want_loglik=want_ll)
            torch.cuda.synchronize()
            assert float(junk[-1]) == float(junk[-1])
            assert torch.equal(a, b), it
            if want_ll:
                assert np.array_equal(ll_a, ll_b)
    finally:
        L.lmosem_events_free(ev)
        c4.close()


def test_autotune_keeps_results(tiny, dev):
    L, ctx, mu = tiny["L"], tiny["ctx"], tiny["mu"]
    start = torch.as_tensor((mu > 0).astype(np.float32), device=dev)
    ev = L.lmosem_events_load(ctx.handle, tiny["evd"])
    try:
        a = start.clone()
        L.lmosem_iterate(ctx.handle, ev, 3, a)
        tile, chunk, graphs = L.lmosem_autotune(ctx.handle, ev)
        assert tile in (8, 16, 32) and chunk in (64, 128, 256, 512, 1024, 2048, 4096) and graphs in (0, 1)
        b = start.clone()
        L.lmosem_iterate(ctx.handle, ev, 3, b)
        torch.cuda.synchronize()
        np.testing.assert_allclose(b.cpu().numpy(), a.cpu().numpy(), rtol=2e-6, atol=1e-12)
    finally:
        L.lmosem_events_free(ev)


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_pixel_tile_plans_match_oracle(brain, dev, tmp_path, monkeypatch, waves):
    # the autotuner's first choice is stored in the tuning cache; the stored
    # line is then rewritten to each pixel tile (64, 128, 256 emission pixels
    # per forward workgroup), read back by the autotuner of a fresh set, and
    # that plan's 10 iterations compared with the oracle
    L, m, ctx, w = brain["L"], brain["m"], brain["ctx"], brain["w"]
    ev = synth.workload_events(w, realisation=6, n_events=3000)
    evd = L.events_to_device(ev, dev)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LMOSEM_TUNE_CACHE", str(cache))
    first = L.lmosem_events_load(ctx.handle, evd)
    try:
        tile, chunk, graphs = L.lmosem_autotune(ctx.handle, first)
        plan = L.lmosem_evset_plan(first)
        assert (plan["event_tile"], plan["chunk_rows"], plan["graphs"]) == (tile, chunk, graphs)
        assert plan["pixel_waves"] in (1, 2, 4)
    finally:
        L.lmosem_events_free(first)
    key, fields = cache.read_text().splitlines()[-1].split("|")
    ev_tile, ch, gr, _ = (int(x) for x in fields.split())
    cache.write_text(f"{key}|{ev_tile} {ch} {gr} {waves}\n")
    evs = L.lmosem_events_load(ctx.handle, evd)
    try:
        L.lmosem_autotune(ctx.handle, evs)
        assert L.lmosem_evset_plan(evs) == {"event_tile": ev_tile, "pixel_waves": waves, "chunk_rows": ch,
                                            "graphs": gr}
        img = torch.as_tensor((brain["mu"] > 0).astype(np.float32), device=dev).contiguous()
        L.lmosem_iterate(ctx.handle, evs, 10, img)
        torch.cuda.synchronize()
        got = img.cpu().numpy().ravel()[m.support]
    finally:
        L.lmosem_events_free(evs)
    H = m.system_matrix(ev)
    ns = brain["g"]["n_subsets"]
    sens = np.stack([m.sensitivity(i) for i in range(ns)])
    f_ref, _ = O.os_lm_mlem(H, ev["angle"], sens, 10, np.ones(len(m.support)), ns)
    ok, worst = _image_ok(got, f_ref)
    assert ok, worst


def test_tuning_cache_lines_without_a_pixel_tile(brain, dev, tmp_path, monkeypatch):
    # a cached choice written before the pixel tile was searched (three
    # fields) is still used, with the context's own pixel tile
    L, ctx, w = brain["L"], brain["ctx"], brain["w"]
    ev = synth.workload_events(w, realisation=7, n_events=2000)
    evd = L.events_to_device(ev, dev)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LMOSEM_TUNE_CACHE", str(cache))
    first = L.lmosem_events_load(ctx.handle, evd)
    try:
        L.lmosem_autotune(ctx.handle, first)
        default_waves = L.lmosem_evset_plan(first)["pixel_waves"]
    finally:
        L.lmosem_events_free(first)
    key = cache.read_text().splitlines()[-1].split("|")[0]
    cache.write_text(f"{key}|16 512 0\n")
    evs = L.lmosem_events_load(ctx.handle, evd)
    try:
        assert L.lmosem_autotune(ctx.handle, evs) == (16, 512, 0)
        plan = L.lmosem_evset_plan(evs)
        assert plan["event_tile"] == 16 and plan["chunk_rows"] == 512 and plan["graphs"] == 0
        assert plan["pixel_waves"] == min(4, (len(brain["m"].support) + 63) // 64)
        assert default_waves in (1, 2, 4)
    finally:
        L.lmosem_events_free(evs)


@pytest.mark.parametrize("chunk", [64, 4096])
def test_backprojection_chunk_extremes_match_oracle(brain, dev, tmp_path, monkeypatch, chunk):
    # the smallest and largest backprojection chunks the autotuner may pick,
    # forced through the tuning cache: 64 rows splits each subset's 250 rows
    # into four chunks summed by the update, 4096 leaves one; 10 iterations
    # of OS-LM-MLEM against the oracle
    L, m, ctx, w = brain["L"], brain["m"], brain["ctx"], brain["w"]
    ev = synth.workload_events(w, realisation=8, n_events=2000)
    evd = L.events_to_device(ev, dev)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LMOSEM_TUNE_CACHE", str(cache))
    first = L.lmosem_events_load(ctx.handle, evd)
    try:
        L.lmosem_autotune(ctx.handle, first)
    finally:
        L.lmosem_events_free(first)
    key = cache.read_text().splitlines()[-1].split("|")[0]
    cache.write_text(f"{key}|8 {chunk} 0 1\n")
    evs = L.lmosem_events_load(ctx.handle, evd)
    try:
        assert L.lmosem_autotune(ctx.handle, evs) == (8, chunk, 0)
        assert L.lmosem_evset_plan(evs)["chunk_rows"] == chunk
        img = torch.as_tensor((brain["mu"] > 0).astype(np.float32), device=dev).contiguous()
        L.lmosem_iterate(ctx.handle, evs, 10, img)
        torch.cuda.synchronize()
        got = img.cpu().numpy().ravel()[m.support]
    finally:
        L.lmosem_events_free(evs)
    H = m.system_matrix(ev)
    ns = brain["g"]["n_subsets"]
    sens = np.stack([m.sensitivity(i) for i in range(ns)])
    f_ref, _ = O.os_lm_mlem(H, ev["angle"], sens, 10, np.ones(len(m.support)), ns)
    ok, worst = _image_ok(got, f_ref)
    assert ok, worst

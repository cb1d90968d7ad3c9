"""The task evaluation of Sec. 3 on the GPU pipeline: noise realisations of
the 64x64 brain reconstructed as one batch through the prepared-set path
(the bench's launch configuration), taken through the task measures
(``paper_2002_12471_amd.tasks``: striatal uptake, its normalised RMSE over
the realisations after every iteration, region-to-background ratios and the
image NRMSE), against the same measures of the FP64 oracle's reconstructions
of the same events.

Tolerances: the images per pixel as in test_gpu_parity; the uptake NRMSE
within 5e-4 (absolute, on a value of order 0.1-0.5: per-pixel agreement of
1e-3 moves a region mean by far less); ratios and image NRMSE within 1e-3
relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
import synth  # noqa: E402

R, N_EV, N_IT = 6, 5000, 10


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def test_task_measures_from_gpu_batch_match_oracle(dev):
    L = _lib()
    from paper_2002_12471_amd import tasks
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    parts = [synth.workload_events(w, realisation=200 + r, n_events=N_EV) for r in range(R)]
    ev = {k: np.concatenate([p[k] for p in parts]) for k in ("angle", "u_bin", "energy")}
    offsets = [0] + list(np.cumsum([N_EV] * R))
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        sens_gpu = ctx.sensitivity(-1).double().cpu().numpy()
        evs = L.lmosem_events_load(ctx.handle, L.events_to_device(ev, dev), offsets)
        L.lmosem_autotune(ctx.handle, evs)
        img = torch.as_tensor(np.broadcast_to((mu > 0).astype(np.float32), (R,) + mu.shape).copy(), device=dev)
        gpu = []
        for _ in range(N_IT):
            L.lmosem_iterate(ctx.handle, evs, 1, img, n_real=R)
            gpu.append(img.double().cpu().numpy())
        L.lmosem_events_free(evs)
    finally:
        ctx.close()

    m = O.OracleModel(g, mu)
    ns = int(g["n_subsets"])
    sens_sub = np.stack([m.sensitivity(i) for i in range(ns)])
    sens_orc = m.to_image(m.sensitivity(-1))
    orc = [np.zeros((R,) + mu.shape) for _ in range(N_IT)]
    for r, p in enumerate(parts):
        H = m.system_matrix(p)
        f = np.ones(len(m.support))
        for t in range(N_IT):
            f, _ = O.os_lm_mlem(H, p["angle"], sens_sub, 1, f, ns)
            orc[t][r] = m.to_image(f)

    # the images themselves, per pixel, after the last iteration
    for r in range(R):
        ref = orc[-1][r].ravel()[m.support]
        got = gpu[-1][r].ravel()[m.support]
        tol = np.where(ref >= 1e-2 * ref.max(), 1e-3 * ref, 1e-5 * ref.max())
        assert np.all(np.abs(got - ref) <= tol), r

    caud, put = synth.striatal_masks(w.geom)
    brain = act > 0
    bg = brain & ~caud & ~put
    truth = act.astype(np.float64)
    counts = [N_EV] * R
    for name, reg in (("caudate", caud & brain), ("putamen", put & brain)):
        a = [tasks.uptake_nrmse(gpu[t], reg, truth, counts, sens_gpu) for t in range(N_IT)]
        b = [tasks.uptake_nrmse(orc[t], reg, truth, counts, sens_orc) for t in range(N_IT)]
        print(f"{name} uptake NRMSE by iteration, GPU: {' '.join(f'{x:.4f}' for x in a)}")
        print(f"{name} uptake NRMSE by iteration, oracle: {' '.join(f'{x:.4f}' for x in b)}")
        np.testing.assert_allclose(a, b, rtol=0, atol=5e-4)
        np.testing.assert_allclose(tasks.region_ratios(gpu[-1], reg, bg), tasks.region_ratios(orc[-1], reg, bg),
                                   rtol=1e-3)
    np.testing.assert_allclose(tasks.image_nrmse(gpu[-1], truth, brain), tasks.image_nrmse(orc[-1], truth, brain),
                               rtol=1e-3)

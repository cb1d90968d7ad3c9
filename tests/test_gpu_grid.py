"""Non-square and odd-sized grids.  A 17 x 13 grid holds the same pixel
centres as the middle 13 rows of a 17 x 17 grid (both are centred on the
rotation axis), so with the extra rows at mu = 0 and no activity the two
contexts describe the same object: sensitivities, per-event means and
reconstructions must agree (the oracle handles square grids only; this pins
the rectangular indexing against the square case it already checks)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


@pytest.mark.parametrize("scatter_model", [1, 0])
def test_rectangular_grid_equals_padded_square_grid(scatter_model):
    L = _lib()
    dev = torch.device("cuda:0")
    nx, ny, pad, dx = 17, 13, 2, 0.8
    sq = synth.Geometry(nx, nx, dx, 20, 0.8, 16, n_subsets=4)
    rect = synth.Geometry(nx, ny, dx, 20, 0.8, 16, n_subsets=4)
    X, Y = synth.phantoms.pixel_centres(nx, nx, dx)
    mu_sq = np.where((X / 6.0) ** 2 + (Y / 4.4) ** 2 <= 1.0, 0.15, 0.0).astype(np.float32)
    act_sq = np.where((X / 5.0) ** 2 + (Y / 3.6) ** 2 <= 1.0, 1.0, 0.0).astype(np.float32)
    act_sq[np.hypot(X - 1.6, Y + 0.8) < 1.2] = 4.0
    assert not mu_sq[:pad].any() and not mu_sq[-pad:].any()
    mu_rect, act_rect = mu_sq[pad:nx - pad].copy(), act_sq[pad:nx - pad].copy()
    ev = synth.generate_events(sq, act_sq, mu_sq, 4000, 123)
    evd = L.events_to_device(ev, dev)
    out = {}
    for name, geom, mu, act in (("sq", sq, mu_sq, act_sq), ("rect", rect, mu_rect, act_rect)):
        ctx = L.Context(dict(geom.as_dict(), scatter_model=scatter_model), torch.as_tensor(mu, device=dev))
        try:
            sens = ctx.sensitivity(1).cpu().numpy()
            mean = ctx.forward(evd, torch.as_tensor(act, device=dev)).cpu().numpy()
            img = ctx.reconstruct(evd, 5).cpu().numpy()
        finally:
            ctx.close()
        if name == "sq":
            sens, img = sens[pad:nx - pad], img[pad:nx - pad]
        out[name] = (sens, mean, img)
    (s0, m0, i0), (s1, m1, i1) = out["sq"], out["rect"]
    np.testing.assert_allclose(s1, s0, rtol=1e-5, atol=1e-7 * s0.max())
    live = m0 > 0
    assert live.sum() > 3900
    np.testing.assert_allclose(m1[live], m0[live], rtol=1e-5)
    np.testing.assert_allclose(i1, i0, rtol=1e-4, atol=1e-5 * i0.max())

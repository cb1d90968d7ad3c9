"""The allocation-free forward projection (lmosem_forward_noalloc) against
lmosem_forward through the C ABI: the same per-event means, bit for bit, on
two calls in a row whose second input is smaller (the scratch array keeps the
first call's contents), on the 64x64 brain (several forward chunks for the
larger call) and on the tiny disk; and its refusals, which the host decides
before any device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def _lib():
    from paper_2002_12471_amd import lmosem as L
    return L


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,sizes", [("brain64", (60_000, 7_001)), ("tiny", (5_000, 37))])
def test_noalloc_forward_equals_forward(dev, name, sizes):
    L = _lib()
    w = synth.workload(name)
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ctx = L.Context(g, torch.as_tensor(mu, device=dev))
    try:
        ctx.sensitivity(-1)   # the path tables are built at the first list-mode call
        img = torch.as_tensor(act, device=dev)
        before = ctx.stats()
        for k, n in enumerate(sizes):
            print(f"{name}: call {k} with {n} events", flush=True)
            ev = L.events_to_device(synth.workload_events(w, realisation=40 + k, n_events=n), dev)
            ref = ctx.forward(ev, img)
            got = torch.full_like(ref, -1.0)
            L.lmosem_forward_noalloc(ctx.handle, ev, img, got)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), float((got - ref).abs().max())
        after = ctx.stats()
        # both calls count the same terms
        assert (after["inner_terms"] - before["inner_terms"]) % 2 == 0
    finally:
        ctx.close()


def test_noalloc_forward_refusals(dev):
    L = _lib()
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    mu_d = torch.as_tensor(mu, device=dev)
    img = torch.as_tensor(act, device=dev)
    ev = L.events_to_device(synth.workload_events(w, n_events=100), dev)
    out = torch.empty(100, device=dev)
    ctx = L.Context(g, mu_d)
    try:
        with pytest.raises(L.LmosemError) as ei:      # tables not built yet
            L.lmosem_forward_noalloc(ctx.handle, ev, img, out)
        assert ei.value.status == L.EINVAL
        ctx.sensitivity(-1)
        L.lmosem_forward_noalloc(ctx.handle, ev, img, out)
        # more events than the scratch array holds: refused from the sizes
        # alone (the arrays are never read)
        big = {k: v[:1].repeat(3_000_000).contiguous() for k, v in ev.items()}
        with pytest.raises(L.LmosemError) as ei:
            L.lmosem_forward_noalloc(ctx.handle, big, img, torch.empty(3_000_000, device=dev))
        assert ei.value.status == L.ENOMEM
        # the context stays usable
        L.lmosem_forward_noalloc(ctx.handle, ev, img, out)
    finally:
        ctx.close()
    sctx = L.Context(dict(g, scatter_model=2), mu_d)
    try:
        sctx.sensitivity(-1)
        with pytest.raises(L.LmosemError) as ei:
            L.lmosem_forward_noalloc(sctx.handle, ev, img, out)
        assert ei.value.status == L.ENOTSUP
    finally:
        sctx.close()

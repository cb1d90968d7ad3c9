"""Emission set from a crude binned OS-MLEM image (orchestration only).

The work of every list-mode iteration grows with the number of estimated
pixels, so the estimate can be confined to a rough object boundary found by
a quick binned reconstruction (Sec. 2.2).  This module chains the library
calls: events binned over the whole acceptance window, a few binned OS-MLEM
iterations on a context that never builds the list-mode path table, and the
boundary kernel (threshold relative to the image maximum, widened by a disc,
kept inside mu > 0).  The mask it returns is meant for
``Context(..., emission=mask)``.
"""
from __future__ import annotations

import torch

from . import lmosem as L


def binned_boundary(geom: dict, mu: torch.Tensor, events: dict, n_pos: int = 64, n_iters: int = 4,
                    threshold: float = 0.05, margin_px: int = 1,
                    stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """[ny][nx] float32 0/1 mask on mu's device: mu > 0 pixels within
    margin_px of a pixel whose binned OS-MLEM value (n_pos position bins,
    one energy bin spanning the window, n_iters iterations) reaches
    threshold x its maximum."""
    edges = [geom["win_lo_kev"], geom["win_hi_kev"]]
    ctx = L.Context(geom, mu, stream)
    try:
        counts = torch.empty(int(geom["n_angles"]) * n_pos, device=mu.device)
        L.lmosem_bin_events(ctx.handle, events, n_pos, edges, counts)
        crude = torch.empty_like(mu)
        L.lmosem_binned_reconstruct(ctx.handle, n_pos, edges, counts, n_iters, crude)
        mask = torch.empty_like(mu)
        L.lmosem_emission_mask(ctx.handle, crude, threshold, margin_px, mask)
    finally:
        ctx.close()
    return mask

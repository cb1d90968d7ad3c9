"""Benchmark: list-mode events/s per OSEM subset update on one MI355X.

Default workload (brain64): 64x64 pixels of 0.4 cm, skull ring (mu 0.25/cm)
around brain (mu 0.15/cm, activity 1) with caudate/putamen ellipses at 8:1
uptake, 128 detector bins of 0.2 cm x 120 angles over 360 degrees, 200k
list-mode events over 100-175 keV from the Monte-Carlo acquisition, 8
subsets.  --workload batch_tiny runs 64 realisations of the 16x16 disk with
log-uniform 50k-500k events each in one batch; --workload brain128 runs the
same head at 128x128 pixels of 0.2 cm with 2M events per realisation over
90-175 keV and 16 subsets.

One step is one global OS-LM-MLEM iteration: every subset update (forward
projection, per-event means, backprojection, multiplicative update) over all
events of all realisations, inputs resident in HBM.  --cache-rows keeps the
system rows after a first (untimed) iteration, so that timed iterations read
them from HBM instead of recomputing them; that line is a separate,
HBM-bound measurement.  value = events per
second = events / step time (the sum over subsets of J_i over the sum of
t_i).  Table build, event ingest, autotuning and the CPU baseline are timed
outside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "list-mode events/s per OSEM subset update; surrogate vs exact at stated error"

# MI355X: 256 CUs at 2.4 GHz.  FP32 FMA issue: 128 lanes per CU and clock
# (the published 157.3 TFLOP/s FP32 vector = 256 x 2.4e9 x 128 x 2 flops;
# non-packed FMAs reach past 64 by dual issue: 88-94 lane-ops/clk/CU measured
# with register operands).  v_exp_f32 (and v_rcp_f32): 32 lanes per CU and
# clock, a quarter of that (30 measured), and it does not overlap the FMAs
# (measured: an exp2 and two independent FMAs take the sum of their times).
N_CU, CLK = 256, 2.4e9
FMA_LANES, TRANS_LANES = 128, 32
FLOPS_PER_TERM = 5      # FMA (2) + exp2 (1) + FMA (2)
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
FP32_PUBLISHED_FLOPS = 157.3e12   # MI355X FP32 vector (128 FMA lanes per CU and clock)


WORKLOAD_TEXT = {
    "tiny": "tiny: 16x16 disk of 0.8 cm px, 16 bins x 16 angles, 5000 events 100-175 keV, 1 subset",
    "brain64": "brain64: 64x64 px of 0.4 cm, 128 bins x 120 angles, 200k events 100-175 keV, "
               "8 subsets, exact first-order scatter path",
    "batch_tiny": "batch_tiny: 64 realisations of the 16x16 disk (0.8 cm px, 16 bins x 16 angles), "
                  "50k-500k events each (log-uniform), 1 subset, one launch per kernel for all",
    "brain128": "brain128: 128x128 px of 0.2 cm, 256 bins x 120 angles, 2M events per realisation "
                "90-175 keV, 16 subsets, exact first-order scatter path",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mix_peak_terms_per_s():
    # CU-clocks per lane-term: two FMAs at FMA_LANES and one exp2 at TRANS_LANES
    return N_CU * CLK / (2.0 / FMA_LANES + 1.0 / TRANS_LANES)


def profiled_traffic(event_tile, pixel_tile, workload, cached=False):
    """HBM bytes per launch of the dominant kernel (the forward projection at
    this event and pixel tile, or with cached rows the row-dot kernel) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None if the kernel source
    changed since the counters were taken or the case was not profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_row_dot_{workload}_cached.md" if cached else f"k_forward_{workload}.md")
    src = os.path.join(ROOT, "paper_2002_12471_amd", "csrc", "osem.hip")
    try:
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                fields[k.split(" (")[0].strip()] = v.strip()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        key = ("traffic_bytes_per_launch_row_dot" if cached
               else f"traffic_bytes_per_launch_ev{event_tile}_px{pixel_tile}")
        if fields.get("source_sha256") != sha or key not in fields:
            return None
        return float(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def binned_boundary(L, torch, np, g, mu_d, act, evd, stream, n_pos=64, n_iters=4, threshold=0.05, margin=1):
    """Emission set from a crude binned OS-MLEM image (the package's
    boundary module), with a summary: sizes, front-end time and the share of
    the true activity it holds."""
    from paper_2002_12471_amd.boundary import binned_boundary as boundary
    torch.cuda.synchronize()
    t0 = time.time()
    mask = boundary(g, mu_d, evd, n_pos, n_iters, threshold, margin, stream)
    torch.cuda.synchronize()
    t_front = time.time() - t0
    mk = mask.cpu().numpy() > 0
    n_sup = int((mu_d.cpu().numpy() > 0).sum())
    return mask, {"from": f"binned OS-MLEM ({n_pos} position bins, whole window, {n_iters} iterations)",
                  "threshold": threshold, "margin_px": margin, "n_emission": int(mk.sum()), "n_support": n_sup,
                  "activity_pixels_inside": float(mk[act > 0].mean()),
                  "front_end_ms": t_front * 1e3}


def cpu_baseline(w, act, mu, ev, n_sample=2048, seed=11):
    """The FP64 oracle on the host cores: one subset update (system rows,
    forward, backprojection, update) for a seeded sample of subset 0's events."""
    import numpy as np
    import oracle as O
    g = w.geom.as_dict()
    if w.name == "brain128":
        n_sample = min(n_sample, 256)
    t0 = time.time()
    m = O.OracleModel(g, mu)
    t_model = time.time() - t0
    sel = np.nonzero(ev["angle"] % g["n_subsets"] == 0)[0]
    idx = np.sort(np.random.default_rng(seed).choice(sel, min(n_sample, sel.size), replace=False))
    sub = {k: ev[k][idx] for k in ("angle", "u_bin", "energy")}
    f = np.ones(len(m.support))
    sens = m.sensitivity(0)
    t0 = time.time()
    H = m.system_matrix(sub)
    O.subset_update(H, f, sens)
    dt = time.time() - t0
    return {"value": len(idx) / dt, "unit": "events/s", "cores": m.n_threads, "host_cpus": os.cpu_count(),
            "kind": "oracle",
            "sample": f"{len(idx)} seeded events of subset 0 of {w.name}: FP64 system rows, "
                      f"forward, backprojection and update ({dt:.1f} s wall on {m.n_threads} "
                      f"threads; model build {t_model:.1f} s not counted)"}


# The fused network per (event, pixel) pair: 384 GELUs evaluated two at a
# time, twelve instructions per pair of them (the conversion from the FP32
# accumulators, the sigmoid factor's polynomial in packed fp16 with its
# clamp, two mixed-precision products and the bf16 rounding; no
# transcendental): 2,304 lane-ops.  These issue at 64 lanes per CU and clock
# (each kind measured at 54-58; no dual issue), 36 CU-clocks per pair.  The MFMA work (67,840 useful flops per pair, the output row
# included; 77,824 as issued, with layer 1's inputs padded to 32 and the
# output row's fifteen zero rows) takes 19.1 CU-clocks at 2.5 PFLOP/s.
MLP_PK_OPS, MLP_PK_LANES = 192 * 12, 64
MLP_PEAK_PAIRS = N_CU * CLK / (MLP_PK_OPS / MLP_PK_LANES)
# The bound the measured issue rates set: the kernel's whole vector-ALU work
# per pair as the SQ counters count it (2,436 lane-ops: the GELUs plus the
# input words, the output and the addressing) and its 4.75 MFMA issues, one
# issue slot of 64 lanes each, at the 57 lanes per clock and CU that every
# instruction kind the GELU uses was probed to issue at.
MLP_VALU_LANE_OPS, MLP_MFMA_ISSUES, MLP_PROBED_LANES = 2436, 4.75, 57
MLP_PRACTICAL_PAIRS = N_CU * CLK / ((MLP_VALU_LANE_OPS + 64 * MLP_MFMA_ISSUES) / MLP_PROBED_LANES)
MLP_FLOPS_PER_PAIR = 2 * (8 * 128 + 2 * 128 * 128 + 128)
BF16_PEAK_FLOPS = 2.5e15   # MI355X dense bf16 MFMA
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def stored_oracle_means(name, ev, np):
    """Per-event means at the true activity that the FP64 oracle wrote for
    these events (tests/golden/make_golden.py), with the event indices they
    belong to; None when the file is absent or was made from other events."""
    path = os.path.join(GOLDEN_DIR, name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    sums = np.array([len(ev["angle"]), float(np.sum(ev["angle"].astype(np.int64))),
                     float(np.sum(ev["u_bin"].astype(np.float64))), float(np.sum(ev["energy"].astype(np.float64)))])
    if not np.array_equal(sums, d["event_checksums"]):
        return None
    return d["index"], d["means"]


def train_surrogate(L, torch, np, synth, large, epochs, dev):
    """Train the scatter network on random elliptical maps (the last 32 held
    out) with the library's own kernels; returns (network, training summary)."""
    from paper_2002_12471_amd import surrogate as S
    wm = synth.workload("surrogate_maps_128" if large else "surrogate_maps")
    gm = wm.geom.as_dict()
    rng = np.random.default_rng(synth.seed_for(wm))
    n_maps, per_map = wm.extra["n_maps"], wm.extra["n_samples"] // wm.extra["n_maps"]
    maps = [synth.random_ellipse_map(wm.geom, rng, wm.extra.get("shell_prob", 0.0), wm.extra.get("body", (0.4, 0.9)))
            for _ in range(n_maps)]
    draws = [synth.surrogate_sample_inputs(wm.geom, m, per_map, rng) for m in maps]
    log(f"surrogate samples: {n_maps} maps x {per_map} ({wm.geom.nx}x{wm.geom.ny} grid)")
    torch.cuda.synchronize()
    t0 = time.time()
    X, t = S.make_samples(gm, maps[:-32], draws[:-32], dev)
    Xv, tv = S.make_samples(gm, maps[-32:], draws[-32:], dev)
    torch.cuda.synchronize()
    t_samples = time.time() - t0
    log(f"training ({t_samples:.1f} s of samples)")
    t0 = time.time()
    net, loss = S.train(synth.mlp_init_params(synth.seed_for(wm, 1)), X, t, rng.permutation(X.shape[0]),
                        batch=4096, epochs=epochs, lr=2e-3, lr_decay=0.93)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    info = {"samples": int(X.shape[0]), "maps": n_maps - 32, "grid": f"{wm.geom.nx}x{wm.geom.ny} px of "
            f"{wm.geom.pixel_cm} cm", "epochs": epochs, "loss_first": float(loss[0]), "loss_last": float(loss[-1]),
            "heldout_mse": S.mse(net, Xv, tv), "sample_s": t_samples, "train_s": t_train}
    return net, info


def surrogate_compare(L, torch, np, synth, large, epochs, steps, warm, full):
    """The learned scatter path against the exact one on the same GPU and the
    same events: on the tiny disk (maps on its 16x16 grid) or on the 128x128
    brain (maps on that grid; per-event errors on a seeded 64k subsample of
    its 2M events).  Event-mean errors at the true activity against the exact
    FP32 path and against the FP64 oracle's stored means, events/s of whole
    iterations for both paths, and the fused network kernel timed inside
    them.  With full, also the images after 10 iterations (and the striatal
    uptake on the brain)."""
    dev = torch.device("cuda:0")
    net, train = train_surrogate(L, torch, np, synth, large, epochs, dev)
    w = synth.workload("brain128" if large else "tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev_np = synth.workload_events(w)
    ev = L.events_to_device(ev_np, dev)
    J = int(ev["angle"].numel())
    stored = stored_oracle_means("brain128_means.npz" if large else "tiny_means.npz", ev_np, np)
    if large:   # per-event errors on a seeded 64k subsample
        idx = (stored[0] if stored is not None else
               np.sort(np.random.default_rng(synth.seed_for(w, 777)).choice(J, 65536, replace=False)))
    else:
        idx = stored[0] if stored is not None else np.arange(J)
    ev_eval = L.events_to_device({k: ev_np[k][idx] for k in ("angle", "u_bin", "energy")}, dev)
    mu_d = torch.as_tensor(mu, device=dev)
    ctxs = {"exact": L.Context(g, mu_d), "primary": L.Context(dict(g, scatter_model=0), mu_d),
            "surrogate": L.Context(dict(g, scatter_model=2), mu_d)}
    L.lmosem_set_surrogate(ctxs["surrogate"].handle, net)
    img = torch.as_tensor(act, device=dev)
    log("event means")
    means = {k: c.forward(ev_eval, img).double() for k, c in ctxs.items()}

    def mean_rel(a, b):   # over events with a positive reference mean (the rest are skipped by every path)
        ok = b > 0
        return float(((a[ok] - b[ok]).abs() / b[ok]).mean())
    rel = {k: mean_rel(means[k], means["exact"]) for k in ("surrogate", "primary")}
    rel_orc = None
    if stored is not None:
        o = torch.as_tensor(stored[1], device=dev)
        rel_orc = {k: mean_rel(means[k], o) for k in ("exact", "surrogate", "primary")}
    extra = {}
    if full:
        log("reconstructions")
        recon = {k: c.reconstruct(ev, 10).double() for k, c in ctxs.items()}
        ref = recon["exact"]
        extra["image_rel_l2_vs_exact_recon_iter10"] = {
            k: float(((recon[k] - ref) ** 2).sum().sqrt() / (ref ** 2).sum().sqrt()) for k in ("surrogate", "primary")}
        rel10 = {}
        for k in ("surrogate", "primary"):
            m_e = ctxs["exact"].forward(ev_eval, recon["exact"].float().contiguous()).double()
            m_k = ctxs[k].forward(ev_eval, recon["exact"].float().contiguous()).double()
            rel10[k] = mean_rel(m_k, m_e)
        extra["mean_rel_event_error_at_iter10_image"] = rel10
        if large:   # striatal uptake after 10 iterations: region mean over the brain background mean
            caud, put = synth.striatal_masks(w.geom)
            bg = (act > 0) & ~caud & ~put
            bg_t = torch.as_tensor(bg, device=dev)
            uptake = {}
            for name, m in (("caudate", caud), ("putamen", put)):
                mt = torch.as_tensor(m & (act > 0), device=dev)
                uptake[name] = {"truth": float(act[m & (act > 0)].mean() / act[bg].mean()),
                                **{k: float(recon[k][mt].mean() / recon[k][bg_t].mean())
                                   for k in ("exact", "surrogate", "primary")}}
            extra["striatal_uptake_ratio_iter10"] = uptake
    # throughput: whole iterations, inputs resident
    rates, stream = {}, torch.cuda.current_stream(dev)
    net_stats = None
    for k in ("exact", "surrogate"):
        log(f"timing {k}")
        c = ctxs[k]
        evs = L.lmosem_events_load(c.handle, ev)
        L.lmosem_autotune(c.handle, evs)
        x = torch.as_tensor((mu > 0).astype(np.float32), device=dev).contiguous()
        for _ in range(warm):
            L.lmosem_iterate(c.handle, evs, 1, x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            L.lmosem_iterate(c.handle, evs, 1, x)
        e1.record(stream)
        torch.cuda.synchronize()
        rates[k] = J * steps / (e0.elapsed_time(e1) * 1e-3)
        if k == "surrogate":
            # the network kernel inside the same iterations, each launch timed
            # with HIP events on the context stream
            L.lmosem_set_timing(c.handle, True)
            for _ in range(max(1, steps // 2)):
                L.lmosem_iterate(c.handle, evs, 1, x)
            net_stats = L.lmosem_get_stats(c.handle)
            L.lmosem_set_timing(c.handle, False)
        L.lmosem_events_free(evs)
    pairs_live = net_stats["network_pairs"] / max(1e-12, net_stats["network_ms"] * 1e-3)
    peak_pairs = MLP_PEAK_PAIRS
    table = {k: ctxs[k].stats()["table_bytes"] for k in ("exact", "surrogate")}
    n_sup = int(ctxs["exact"].stats()["n_support"])
    for c in ctxs.values():
        c.close()
    target = ("the 128x128 brain (2M events, 16 subsets; event errors on a seeded 64k subsample)" if large
              else "the tiny disk (5000 events, 1 subset)")
    out = {
        "workload": f"MLP 8-128-128-128-1 GELU, bf16 MFMA with FP32 accumulation, trained on {train['samples']} "
                    f"far-field samples from {train['maps']} random elliptical maps (mu 0.1-0.3/cm, {train['grid']}), "
                    f"near field exact, used in LM-OSEM on {target}",
        "events": J, "support_pixels": n_sup, "eval_events": int(len(idx)), "steps": steps, "warmup": warm,
        "exact_events_per_s": rates["exact"], "surrogate_events_per_s": rates["surrogate"],
        "surrogate_vs_exact_speed": rates["surrogate"] / rates["exact"],
        "mean_rel_event_error_vs_exact": rel,
        "mean_rel_event_error_vs_oracle": rel_orc,
        **extra,
        "table_bytes": table,
        "network_roofline": {
            "bound": "alu", "kernel": "k_mlp_infer", "achieved": pairs_live / 1e9, "peak": peak_pairs / 1e9,
            "unit": "Gpair/s", "frac": pairs_live / peak_pairs,
            "per_unit": f"one (event, emission pixel) pair = {MLP_PK_OPS} VALU lane-ops for its 384 GELUs "
                        f"(packed fp16 polynomial, bf16 result) at {MLP_PK_LANES} lanes/clk/CU",
            "frac_published_bf16": pairs_live * MLP_FLOPS_PER_PAIR / BF16_PEAK_FLOPS,
            "frac_practical": pairs_live / MLP_PRACTICAL_PAIRS,
            "practical_note": f"{MLP_PRACTICAL_PAIRS / 1e9:.2f} Gpair/s: {MLP_VALU_LANE_OPS} VALU lane-ops and "
                              f"{MLP_MFMA_ISSUES} MFMA issues per pair (SQ counters) at the probed "
                              f"{MLP_PROBED_LANES} lanes/clk/CU",
            "units_per_launch": net_stats["network_pairs"] / max(1, net_stats["network_launches"]),
            "avg_launch_us": net_stats["network_ms"] * 1e3 / max(1, net_stats["network_launches"]),
            "launches_timed": net_stats["network_launches"]},
        "train": train,
    }
    L.lmosem_net_destroy(net)
    return out


def bench_surrogate(args, L, torch, np, synth):
    """--workload surrogate / surrogate128: the comparison on its own line,
    with the images after 10 iterations."""
    large = args.workload == "surrogate128"
    steps, warm = (min(args.steps, 3), min(args.warmup, 1)) if large else (args.steps, args.warmup)
    r = surrogate_compare(L, torch, np, synth, large, args.surrogate_epochs, steps, warm, full=True)
    out = {
        "metric": METRIC, "value": r["surrogate_events_per_s"], "unit": "events/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": r["events"] / r["surrogate_events_per_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32",
        "data": "synthetic (Monte-Carlo list-mode events; random elliptical training maps)",
        "config": {"workload": f"{args.workload}: {r['workload']}", "events": r["events"],
                   "support_pixels": r["support_pixels"]},
        "roofline": r["network_roofline"],
        "surrogate": r,
    }
    print(json.dumps(out), flush=True)


def bench_study(args, L, torch, np, synth):
    """Energy windows, scatter modelling and binning on the brain phantom, the
    paper's experiment design on the synthetic head: R noise realisations of
    the 64x64 brain (200k events each over 100-175 keV), each acceptance
    window's events reconstructed (10 iterations, 8 subsets, all realisations
    in one batch) with first-order scatter modelled and with primary paths
    only, and binned variants (64 position bins, 1-3 energy bins); per
    realisation the caudate and putamen uptakes (normalised RMSE over the
    realisations after every iteration), their ratios to the brain-background
    mean (truth 8) and the image NRMSE against the truth after scaling to the
    truth's brain mean."""
    from paper_2002_12471_amd import tasks
    dev = torch.device("cuda:0")
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    R = args.realisations or 16
    log(f"generating {R} realisations")
    n_ev = args.study_events or w.n_events
    parts = [synth.workload_events(w, realisation=r, n_events=n_ev) for r in range(R)]
    caud, put = synth.striatal_masks(w.geom)
    brain = act > 0
    bg = brain & ~caud & ~put
    masks = {"caudate": caud & brain, "putamen": put & brain}
    truth = act.astype(np.float64)
    mu_d = torch.as_tensor(mu, device=dev)
    rows, events_done, t_recon = [], 0, 0.0
    start = np.broadcast_to((mu > 0).astype(np.float32), (R,) + mu.shape).copy()

    def score(by_iter, counts, sens_all):
        """Task measures of one configuration (paper_2002_12471_amd.tasks)
        from its images after each iteration (by_iter[t][r] = image of
        realisation r after t + 1 iterations): each striatal region's uptake
        NRMSE over the realisations after every iteration (the paper's figure
        of merit), and after the last one each region's ratio to the brain
        background mean (truth 8) and the image NRMSE."""
        imgs = [x.double().cpu().numpy() for x in by_iter]
        sens = sens_all.double().cpu().numpy()
        out = {}
        for k, m in masks.items():
            out[f"{k}_uptake_nrmse_by_iter"] = [tasks.uptake_nrmse(im, m, truth, counts, sens) for im in imgs]
        nrmse = tasks.image_nrmse(imgs[-1], truth, brain)
        out["nrmse_mean"], out["nrmse_std"] = float(nrmse.mean()), float(nrmse.std())
        for k, m in masks.items():
            v = tasks.region_ratios(imgs[-1], m, bg)
            out[f"{k}_ratio_mean"] = float(v.mean())
            out[f"{k}_ratio_std"] = float(v.std())
            out[f"{k}_ratio_bias_pct"] = 100.0 * (float(v.mean()) - 8.0) / 8.0
        return out

    def report(row):
        rows.append(row)
        log(f"{row['window_kev']} keV, {row['model'][:60]}: caudate {row['caudate_ratio_mean']:.2f} +- "
            f"{row['caudate_ratio_std']:.2f}, putamen {row['putamen_ratio_mean']:.2f} +- "
            f"{row['putamen_ratio_std']:.2f}, image nrmse {row['nrmse_mean']:.3f}, uptake nrmse (it 10) "
            f"{row['caudate_uptake_nrmse_by_iter'][-1]:.3f} / {row['putamen_uptake_nrmse_by_iter'][-1]:.3f}")

    sens_whole = None
    for lo in (143.0, 120.0, 100.0):
        sel = [p["energy"] >= lo for p in parts]
        ev = {k: np.concatenate([p[k][m] for p, m in zip(parts, sel)]) for k in ("angle", "u_bin", "energy")}
        sizes = [int(m.sum()) for m in sel]
        offsets = [0] + list(np.cumsum(sizes).astype(int))
        evd = L.events_to_device(ev, dev)
        for model, name in ((1, "first-order scatter"), (0, "primary only")):
            ctx = L.Context(dict(g, win_lo_kev=lo, scatter_model=model), mu_d)
            sens_all = ctx.sensitivity(-1).double()
            if lo == 100.0 and model == 1:
                sens_whole = sens_all
            evs = L.lmosem_events_load(ctx.handle, evd, offsets)
            img = torch.as_tensor(start, device=dev)
            by_iter = []
            torch.cuda.synchronize()
            t0 = time.time()
            for _ in range(10):
                L.lmosem_iterate(ctx.handle, evs, 1, img, n_real=R)
                by_iter.append(img.clone())
            torch.cuda.synchronize()
            t_recon += time.time() - t0
            events_done += 10 * sum(sizes)
            L.lmosem_events_free(evs)
            ctx.close()
            report({"window_kev": [lo, g["win_hi_kev"]], "model": name + ", list mode",
                    "events_per_realisation": int(np.mean(sizes)), **score(by_iter, sizes, sens_all)})
    # binned variants of the whole-spectrum data: 64 position bins (two detector
    # bins each) and 1, 2 or 3 energy bins, first-order scatter modelled
    t_bin = 0.0
    for edges in ([143.0, 175.0], [100.0, 143.0, 175.0], [100.0, 120.0, 143.0, 175.0]):
        ctx = L.Context(dict(g, win_lo_kev=edges[0], scatter_model=1), mu_d)
        sens_all = ctx.sensitivity(-1).double()
        n_pos = g["n_bins"] // 2
        counts = torch.empty(g["n_angles"] * n_pos * (len(edges) - 1), device=dev)
        per_r, n_counts = [], []
        for r in range(R):
            L.lmosem_bin_events(ctx.handle, L.events_to_device(parts[r], dev), n_pos, edges, counts)
            n_counts.append(float(counts.sum()))
            series, prev = [], None
            torch.cuda.synchronize()
            t0 = time.time()
            for _ in range(10):
                img = torch.empty(mu.shape, device=dev)
                L.lmosem_binned_reconstruct(ctx.handle, n_pos, edges, counts, 1, img, init=prev)
                series.append(img)
                prev = img
            torch.cuda.synchronize()
            t_bin += time.time() - t0
            per_r.append(series)
        ctx.close()
        by_iter = [torch.stack([per_r[r][t] for r in range(R)]) for t in range(10)]
        report({"window_kev": [edges[0], edges[-1]], "model": f"first-order scatter, binned: {n_pos} position x "
                f"{len(edges) - 1} energy bins {edges}", "events_per_realisation": int(np.mean(n_counts)),
                **score(by_iter, n_counts, sens_all)})
    # list mode over the whole spectrum with the estimate confined to a crude
    # boundary from each realisation's own binned OS-MLEM (one context per
    # realisation, since the boundary differs)
    gw = dict(g, win_lo_kev=100.0, scatter_model=1)
    per_r, n_em, cover, t_front, t_em = [], [], [], 0.0, 0.0
    for r in range(R):
        evd = L.events_to_device(parts[r], dev)
        mask, info = binned_boundary(L, torch, np, gw, mu_d, act, evd, torch.cuda.current_stream(dev))
        t_front += info["front_end_ms"] * 1e-3
        n_em.append(info["n_emission"])
        cover.append(info["activity_pixels_inside"])
        ctx = L.Context(gw, mu_d, emission=mask)
        evs = L.lmosem_events_load(ctx.handle, evd)
        img = torch.as_tensor(start[0], device=dev)
        series = []
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(10):
            L.lmosem_iterate(ctx.handle, evs, 1, img)
            series.append(img.clone())
        torch.cuda.synchronize()
        t_em += time.time() - t0
        L.lmosem_events_free(evs)
        ctx.close()
        per_r.append(series)
    by_iter = [torch.stack([per_r[r][t] for r in range(R)]) for t in range(10)]
    report({"window_kev": [100.0, g["win_hi_kev"]], "model": "first-order scatter, list mode, estimate confined "
            "to a binned OS-MLEM boundary (64 position bins, 4 iterations, 5% threshold, 1-pixel margin)",
            "events_per_realisation": int(np.mean([len(p["angle"]) for p in parts])),
            **score(by_iter, [len(p["angle"]) for p in parts], sens_whole),
            "emission_pixels_mean": float(np.mean(n_em)), "support_pixels": int((mu > 0).sum()),
            "activity_inside_min": float(np.min(cover)), "front_end_s_per_realisation": t_front / R,
            "reconstruct_s_per_realisation": t_em / R})
    # ordered subsets against plain list-mode MLEM (Sec. 2.2 defines the
    # subsets; Sec. 4 reports close to a fourfold speed-up for 4 subsets):
    # realisation 0 over the whole window; every iterate's full-data
    # log-likelihood sum_j log mean_j - sum_q f_q sens_q from one 1-subset context
    evd = L.events_to_device(parts[0], dev)
    ref = L.Context(dict(gw, n_subsets=1), mu_d)
    sens_all = ref.sensitivity(-1).double()

    def full_ll(img):
        m = ref.forward(evd, img).double()
        return float(torch.log(m[m > 1e-30]).sum() - (img.double() * sens_all).sum())

    curves = {}
    for ns, iters in ((1, 40), (4, 10), (8, 10)):
        ctx = ref if ns == 1 else L.Context(dict(gw, n_subsets=ns), mu_d)
        evs = L.lmosem_events_load(ctx.handle, evd)
        img = torch.as_tensor((mu > 0).astype(np.float32), device=dev)
        ll = [full_ll(img)]
        for _ in range(iters):
            L.lmosem_iterate(ctx.handle, evs, 1, img)
            ll.append(full_ll(img))
        L.lmosem_events_free(evs)
        if ns != 1:
            ctx.close()
        curves[ns] = ll
    ref.close()
    mlem = np.array(curves[1])

    def mlem_iters_to(level):   # first (interpolated) MLEM iteration count reaching the level
        k = int(np.searchsorted(np.maximum.accumulate(mlem), level))
        if k == 0:
            return 0.0
        if k >= len(mlem):
            return float("inf")
        return k - 1 + (level - mlem[k - 1]) / (mlem[k] - mlem[k - 1])

    os_rows = []
    for ns in (4, 8):
        for it in (1, 2, 5, 10):
            need = mlem_iters_to(curves[ns][it])
            fin = bool(np.isfinite(need))   # None: beyond the 40 MLEM iterations run
            os_rows.append({"subsets": ns, "iterations": it, "loglik": curves[ns][it],
                            "mlem_iterations_to_match": need if fin else None, "speedup": need / it if fin else None})
            log(f"OS {ns} subsets, {it} iterations: MLEM needs {need:.1f} iterations ({need / it:.2f}x)")
    out = {
        "metric": METRIC, "value": events_done / t_recon, "unit": "events/s", "n_gpus": 1,
        "steps": 10, "warmup": 0, "ms_per_step": t_recon / 60 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Monte-Carlo list-mode events from the analytic brain phantom)",
        "config": {"workload": f"study: {R} realisations of brain64 ({n_ev} events each over 100-175 keV), "
                               "windows [143,175], [120,175], [100,175] keV, first-order scatter vs primary only, "
                               "list mode and binned (64 position x 1/2/3 energy bins), list mode confined to a "
                               "binned-OS-MLEM boundary, 10 iterations x 8 subsets, "
                               "list-mode realisations batched (value: list-mode events x iterations per second of "
                               "reconstruction, calls included)", "realisations": R,
                   "binned_seconds": t_bin},
        "study": rows,
        "os_vs_mlem": {"loglik_mlem": curves[1], "loglik_os4": curves[4], "loglik_os8": curves[8], "rows": os_rows},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--event-tile", type=int, default=0)
    ap.add_argument("--pixel-tile", type=int, default=0,
                    help="emission pixels per forward workgroup (64-256) with --event-tile; default: the library's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="brain64",
                    choices=["brain64", "tiny", "batch_tiny", "brain128", "surrogate", "surrogate128", "study"])
    ap.add_argument("--surrogate-epochs", type=int, default=40)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="leave out the learned-scatter comparison that the default brain64 line carries")
    ap.add_argument("--cache-rows", action="store_true",
                    help="keep the system rows after the first iteration (HBM-bound iterations; reported apart "
                         "from the default recomputing path)")
    ap.add_argument("--realisations", type=int, default=0,
                    help="realisations for the batched workloads (default: 64 for batch_tiny, 2 for brain128, "
                         "16 for study)")
    ap.add_argument("--emission-from-binned", action="store_true",
                    help="confine the estimate to a crude boundary from a binned OS-MLEM (64 position bins, "
                         "the whole window, 4 iterations, 5%% threshold, 1-pixel margin) before timing")
    ap.add_argument("--study-events", type=int, default=0,
                    help="events per realisation in the study (default: the workload's 200k)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is event sharding with one all-reduce per sub-iteration)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2002_12471_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2002_12471_amd import lmosem as L

    if args.workload in ("surrogate", "surrogate128"):
        bench_surrogate(args, L, torch, np, synth)
        return
    if args.workload == "study":
        bench_study(args, L, torch, np, synth)
        return
    dev = torch.device("cuda:0")
    w = synth.workload(args.workload)
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    log(f"generating events ({args.workload})")
    offsets = None
    if args.workload in ("brain64", "tiny"):
        ev = synth.workload_events(w)
    else:
        if args.workload == "batch_tiny":
            n_real = args.realisations or w.n_real
            sizes = synth.batch_event_counts(w)[:n_real]
        else:
            n_real = args.realisations or 2
            sizes = np.full(n_real, w.n_events)
        parts = [synth.workload_events(w, realisation=r, n_events=int(n)) for r, n in enumerate(sizes)]
        ev = {k: np.concatenate([p[k] for p in parts]) for k in ("angle", "u_bin", "energy")}
        offsets = [0] + list(np.cumsum(sizes).astype(int))
        del parts
    J = len(ev["angle"])
    n_real = 1 if offsets is None else len(offsets) - 1
    evd = L.events_to_device(ev, dev)
    mu_d = torch.as_tensor(mu, device=dev)
    stream = torch.cuda.current_stream(dev)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    emission = None
    if args.emission_from_binned:
        if offsets is not None and len(offsets) > 2:
            sys.exit("--emission-from-binned takes one realisation")
        emission, em_info = binned_boundary(L, torch, np, g, mu_d, act, evd, stream)
        log(f"emission set: {em_info}")
    log("building tables")
    torch.cuda.synchronize()
    t0 = time.time()
    ctx = L.Context(g, mu_d, stream, emission=emission)
    ctx.sensitivity(-1)   # the list-mode tables are built at their first use
    torch.cuda.synchronize()
    t_create = time.time() - t0
    if args.event_tile:
        ctx.set_tuning(args.event_tile, args.pixel_tile)
    t0 = time.time()
    evs = L.lmosem_events_load(ctx.handle, evd, offsets)
    torch.cuda.synchronize()
    t_load = time.time() - t0
    t0 = time.time()
    if not args.event_tile:
        L.lmosem_autotune(ctx.handle, evs)
    t_tune = time.time() - t0
    plan = L.lmosem_evset_plan(evs)
    tile, chunk, graphs = plan["event_tile"], plan["chunk_rows"], plan["graphs"]
    pixel_tile = 64 * plan["pixel_waves"]
    start = np.broadcast_to((mu > 0).astype(np.float32), (n_real,) + mu.shape).copy()
    img = torch.as_tensor(start if n_real > 1 else start[0], device=dev).contiguous()
    t_fill = None
    if args.cache_rows:
        # the first iteration computes and keeps every system row; timed ones reuse them
        L.lmosem_cache_rows(ctx.handle, evs, True)
        torch.cuda.synchronize()
        t0 = time.time()
        L.lmosem_iterate(ctx.handle, evs, 1, img)
        torch.cuda.synchronize()
        t_fill = time.time() - t0

    log("warm-up")
    for _ in range(args.warmup):
        L.lmosem_iterate(ctx.handle, evs, 1, img)
    torch.cuda.synchronize()
    img.copy_(torch.as_tensor(start if n_real > 1 else start[0], device=dev))
    st0 = L.lmosem_get_stats(ctx.handle)

    log(f"timing {args.steps} steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.time()
    e0.record(stream)
    for _ in range(args.steps):
        L.lmosem_iterate(ctx.handle, evs, 1, img)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - w0
    ms_total = e0.elapsed_time(e1)
    st1 = L.lmosem_get_stats(ctx.handle)
    ms_step = ms_total / args.steps
    value = J * args.steps / (ms_total * 1e-3)

    # dominant kernel: forward projection, timed with HIP events on the same stream
    log("timing kernels")
    L.lmosem_set_timing(ctx.handle, True)
    for _ in range(max(2, args.steps // 4)):
        L.lmosem_iterate(ctx.handle, evs, 1, img)
    ks = L.lmosem_get_stats(ctx.handle)
    L.lmosem_set_timing(ctx.handle, False)
    n_it = max(2, args.steps // 4)
    useful_per_iter = (st1["useful_terms"] - st0["useful_terms"]) / args.steps
    computed_per_iter = (st1["inner_terms"] - st0["inner_terms"]) / args.steps
    launches = ks["forward_launches"]
    fwd_s = ks["forward_ms"] * 1e-3 / launches
    useful_per_launch = useful_per_iter * n_it / launches
    achieved_terms = useful_per_launch / fwd_s
    rates = L.lmosem_measure_alu_rates(stream)
    # the ceiling derived from the unit counts and the clock (two FMAs and one
    # quarter-rate exp2 per term); the library's probe of the same mix is
    # reported beside it
    peak_terms = mix_peak_terms_per_s()
    n_qpad = (ctx.stats()["n_emission"] + 63) // 64 * 64
    row_bytes = J * n_qpad * 4 / g["n_subsets"]   # H read per sub-iteration (mean over subsets)
    if args.cache_rows:
        bp_s = ks["backproject_ms"] * 1e-3 / max(1, ks["backproject_launches"])
        roof = {
            "bound": "hbm",
            "kernel": "k_row_dot (event means and their inverses from cached rows)",
            "achieved": row_bytes / fwd_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": row_bytes / fwd_s / 1e9 / HBM_PEAK_GBS,
            "traffic": None if emission is not None else profiled_traffic(tile, pixel_tile, args.workload, cached=True),
            "per_unit": "4 bytes per (event, padded support pixel) of the sub-iteration's rows",
            "units_per_launch": row_bytes / 4,
            "avg_launch_ms": fwd_s * 1e3,
            "backproject_avg_ms": bp_s * 1e3,
            "backproject_gbps": row_bytes / bp_s / 1e9 if bp_s > 0 else None,
            "update_avg_ms": ks["update_ms"] / max(1, ks["update_launches"]),
        }
    else:
        roof = None
    roof = roof or {
        "bound": "alu",
        "kernel": "k_forward (forward projection)",
        "achieved": achieved_terms * FLOPS_PER_TERM / 1e12,
        "peak": peak_terms * FLOPS_PER_TERM / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved_terms / peak_terms,
        "traffic": None if emission is not None else profiled_traffic(tile, pixel_tile, args.workload),
        "per_unit": "one inner term (event, emission pixel, path end with non-zero position "
                    "response) = 2 FMA + 1 exp2 = 5 flops; the kernel evaluates per-path weights "
                    "tabulated once per mu-map in FP64 (w G = 2^(alpha + beta (E - e_c)) times a per-event factor)",
        "peak_derivation": "256 CUs x 2.4 GHz / (2 FMAs at 128 lanes/clk/CU + 1 v_exp_f32 at 32 lanes/clk/CU, "
                           "not overlapped) = 1.31e13 terms/s",
        "frac_published": achieved_terms * FLOPS_PER_TERM / FP32_PUBLISHED_FLOPS,
        "published_peak": FP32_PUBLISHED_FLOPS / 1e12,
        "published_note": "157.3 TFLOP/s FP32 vector is 128 FMA lanes/clk/CU; each term also issues one "
                          "v_exp_f32 at a quarter of that rate, so 5 flops per term cap at 107 of 256 "
                          "flops/clk/CU = 0.42 of the published peak",
        "units_per_launch": useful_per_launch,
        "avg_launch_ms": fwd_s * 1e3,
        "computed_terms_per_launch": computed_per_iter * n_it / launches,
        "measured_rates_per_s": rates,
        "derived_peak_terms_per_s": mix_peak_terms_per_s(),
        "frac_computed_terms": (computed_per_iter * n_it / launches) / fwd_s / peak_terms,
        "backproject_avg_ms": ks["backproject_ms"] / max(1, ks["backproject_launches"]),
        "mean_update_avg_ms": ks["update_ms"] / max(1, ks["update_launches"]),
    }

    out = {
        "metric": METRIC, "value": value, "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Monte-Carlo list-mode events from the analytic %s phantom)" % (
            "brain" if w.phantom == "brain" else "disk"),
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "events": J, "realisations": n_real, "subsets": g["n_subsets"],
                   "support_pixels": int((mu > 0).sum()),
                   **({"emission_set": em_info} if emission is not None else {}),
                   "event_tile": tile, "pixel_tile": pixel_tile, "chunk_rows": chunk, "graphs": bool(graphs),
                   "path": "exact FP32" + (", system rows cached after the first iteration" if args.cache_rows
                                           else "")},
        "roofline": roof,
        "one_time_ms": {"create_tables": t_create * 1e3, "event_ingest": t_load * 1e3,
                        "autotune": t_tune * 1e3,
                        **({"row_cache_fill_iteration": t_fill * 1e3} if t_fill is not None else {})},
        "wall_s_timed": wall,
        "skipped_events": ks["skipped_events"],
    }
    L.lmosem_events_free(evs)
    ctx.close()
    if args.workload == "brain64" and not args.no_surrogate and not args.cache_rows and emission is None:
        # the metric's second half: the learned scatter term against the exact
        # path on the same GPU, at its stated error, on the tiny disk (the
        # network's training grid) and on the 128x128 brain
        del evd
        out["surrogate"] = {
            "tiny": surrogate_compare(L, torch, np, synth, False, args.surrogate_epochs, 10, 2, full=False),
            "brain128": surrogate_compare(L, torch, np, synth, True, args.surrogate_epochs, 2, 1, full=False),
        }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, act, mu, ev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

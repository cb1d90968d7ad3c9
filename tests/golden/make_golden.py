"""Write the stored oracle results that the full-size GPU parity tests read.

Every value written here comes from the FP64 oracle (``oracle/``) applied to
the seeded synthetic inputs of ``synth`` (input generation only); nothing
comes from the GPU library.  The oracle's cost at these sizes (minutes of CPU
per case) is why the results are stored rather than recomputed inside a GPU
test.

  brain64_full_os.npz   the 64x64 brain workload at full size: all 200,000
                        events of realisation 0, 8 subsets, 10 iterations of
                        OS-LM-MLEM (Eq. 7-9) from 1 on the support; the
                        estimate after every iteration and the per-iteration
                        sum of the subsets' Eq. 3 terms.
  brain128_means.npz    the 128x128 brain (2M events of realisation 0, window
                        90-175 keV): per-event means (denominator of Eq. 8) at
                        the true activity for a seeded sample of events.
  tiny_means.npz        the 16x16 disk (5,000 events of realisation 0): the
                        per-event means at the true activity for every event.

Each file also holds checksums of the events it was made from, so that a
test can tell whether the generator still produces the same inputs.

Usage:  python tests/golden/make_golden.py [tiny] [brain64] [brain128] [--n128 N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

BRAIN128_SAMPLE_SEED = 777   # realisation index handed to synth.seed_for for the sample choice


def event_checksums(ev: dict) -> np.ndarray:
    return np.array([len(ev["angle"]), float(np.sum(ev["angle"].astype(np.int64))),
                     float(np.sum(ev["u_bin"].astype(np.float64))),
                     float(np.sum(ev["energy"].astype(np.float64)))])


def brain128_sample(w, n: int) -> np.ndarray:
    """Seeded choice of n event indices among the workload's events."""
    rng = np.random.default_rng(synth.seed_for(w, BRAIN128_SAMPLE_SEED))
    return np.sort(rng.choice(w.n_events, n, replace=False))


def make_brain64(out: str) -> None:
    w = synth.workload("brain64")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    m = O.OracleModel(g, mu)
    t0 = time.time()
    H = m.system_matrix(ev)
    print(f"brain64: {H.shape[0]} system rows in {time.time() - t0:.0f} s on {m.n_threads} threads", flush=True)
    ns = int(g["n_subsets"])
    sens = np.stack([m.sensitivity(i) for i in range(ns)])
    f = np.ones(len(m.support))
    images, ll = [], []
    for _ in range(10):
        f, ll_it = O.os_lm_mlem(H, ev["angle"], sens, 1, f, ns)
        images.append(f.copy())
        ll.append(float(ll_it[0]))
    np.savez_compressed(out, support=m.support, images=np.array(images), loglik=np.array(ll),
                        sens=sens, event_checksums=event_checksums(ev))
    print(f"wrote {out}", flush=True)


def make_brain128(out: str, n: int) -> None:
    w = synth.workload("brain128")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    idx = brain128_sample(w, n)
    sub = {k: ev[k][idx] for k in ("angle", "u_bin", "energy")}
    m = O.OracleModel(g, mu)
    f = act.ravel()[m.support].astype(np.float64)
    means = np.empty(n)
    t0 = time.time()
    step = 512
    for lo in range(0, n, step):
        part = {k: v[lo:lo + step] for k, v in sub.items()}
        means[lo:lo + step] = m.system_matrix(part) @ f
        if (lo // step) % 8 == 0:
            print(f"brain128: {lo + len(part['angle'])} of {n} events, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(out, index=idx, means=means, event_checksums=event_checksums(ev),
                        sample_checksums=event_checksums(sub))
    print(f"wrote {out}", flush=True)


def make_tiny(out: str) -> None:
    w = synth.workload("tiny")
    g = w.geom.as_dict()
    act, mu = synth.phantom(w)
    ev = synth.workload_events(w)
    m = O.OracleModel(g, mu)
    means = m.system_matrix(ev) @ act.ravel()[m.support].astype(np.float64)
    np.savez_compressed(out, index=np.arange(len(means)), means=means, event_checksums=event_checksums(ev),
                        sample_checksums=event_checksums(ev))
    print(f"wrote {out}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=["tiny", "brain64", "brain128"])
    ap.add_argument("--n128", type=int, default=65536)
    a = ap.parse_args()
    if "tiny" in a.cases:
        make_tiny(os.path.join(HERE, "tiny_means.npz"))
    if "brain64" in a.cases:
        make_brain64(os.path.join(HERE, "brain64_full_os.npz"))
    if "brain128" in a.cases:
        make_brain128(os.path.join(HERE, "brain128_means.npz"), a.n128)


if __name__ == "__main__":
    main()

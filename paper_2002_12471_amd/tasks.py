"""Task measures of reconstructed images over noise realisations (Sec. 3:
striatal uptake of the DaT study and its normalised RMSE over realisations,
and the image's normalised RMSE against the truth).

Plain definitions on host arrays: the images come back from the device after
each iteration, and these measures are a few sums per region.

Conventions (the paper gives no formulas for them):
  * the uptake of a region is its mean activity;
  * under the preset-count model every realisation's image carries its own
    count scale (sum_q sens_q f_q equals the realisation's counts after each
    sub-iteration), so the truth a realisation is compared with is the true
    image scaled by counts[r] / sum_q sens_q truth_q;
  * the uptake NRMSE over R realisations is
    sqrt(mean_r (u_r / u_true_r - 1)^2);
  * the ratio of a region is its mean over the background region's mean
    (scale free);
  * the image NRMSE scales the image to the truth's mean over the brain and
    takes ||f - truth|| / ||truth|| over the brain.
"""
from __future__ import annotations

import numpy as np


def count_scales(counts, sens, truth) -> np.ndarray:
    """Per realisation the factor that turns the true image into the one with
    that realisation's counts: counts[r] / sum_q sens_q truth_q."""
    s = float((np.asarray(sens, np.float64) * np.asarray(truth, np.float64)).sum())
    if not s > 0:
        raise ValueError("the true image has no sensitivity-weighted counts")
    return np.asarray(counts, np.float64) / s


def uptake_nrmse(images, region, truth, counts, sens) -> float:
    """Normalised RMSE over realisations of a region's uptake: images[r] is
    realisation r's image, region a boolean mask."""
    region = np.asarray(region, bool)
    if not region.any():
        raise ValueError("empty region")
    u_true = float(np.asarray(truth, np.float64)[region].mean())
    scale = count_scales(counts, sens, truth)
    err = [float(np.asarray(f, np.float64)[region].mean()) / (scale[r] * u_true) - 1.0
           for r, f in enumerate(images)]
    return float(np.sqrt(np.mean(np.square(err))))


def region_ratios(images, region, background) -> np.ndarray:
    """Per realisation the region's mean over the background region's mean."""
    region, background = np.asarray(region, bool), np.asarray(background, bool)
    if not region.any() or not background.any():
        raise ValueError("empty region")
    out = []
    for f in images:
        f = np.asarray(f, np.float64)
        out.append(float(f[region].mean()) / float(f[background].mean()))
    return np.asarray(out)


def image_nrmse(images, truth, brain) -> np.ndarray:
    """Per realisation ||s f - truth|| / ||truth|| over the brain, with s the
    factor that gives f the truth's brain mean."""
    brain = np.asarray(brain, bool)
    t = np.asarray(truth, np.float64)[brain]
    if not (t ** 2).sum() > 0:
        raise ValueError("the truth is zero over the brain")
    out = []
    for f in images:
        fb = np.asarray(f, np.float64)[brain]
        fs = fb * (t.mean() / fb.mean())
        out.append(float(np.sqrt(((fs - t) ** 2).sum() / (t ** 2).sum())))
    return np.asarray(out)

"""Fit of the GELU sigmoid factor used by the network inference kernel
(mlp_infer.h), kept with the kernel so its coefficients can be regenerated.

With s = z/4 on |s| <= 1 and t = s^2 - 1/2, the tanh form's sigmoid factor
sigma(2 sqrt(2/pi) (z + 0.044715 z^3)) is written 1/2 + s P(t), P of degree
6.  The fit minimises the largest |s| times the factor's error (the error of
s times the factor, which the kernel uses) by reweighted least squares, and
rounds the coefficients to fp16 one at a time from the highest, refitting
the lower ones after each rounding.  It prints the coefficients as fp16
literals and the worst error of the kernel's fp16 evaluation against the
tanh form, over every finite fp16 value of s (the kernel forms t with no
clamp, so past |s| = 1 the factor must saturate through its final clamp).
Not used at run time.
"""
import numpy as np

C, A = np.sqrt(2.0 / np.pi), 0.044715
DEG = 6


def factor(s):
    z = 4.0 * s
    return 0.5 * (1.0 + np.tanh(C * (z + A * z ** 3)))


def f16(x):
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def fit():
    s = np.linspace(1e-7, 1.0, 40001)
    t = s * s - 0.5
    target = factor(s) - 0.5
    basis = np.stack([t ** k for k in range(DEG + 1)], 1) * s[:, None]
    fixed = {}
    for top in range(DEG, -1, -1):
        free = [k for k in range(DEG + 1) if k not in fixed]
        y = target - (basis[:, list(fixed)] @ np.array(list(fixed.values())) if fixed else 0.0)
        w = s.copy()
        for _ in range(80):
            c, *_ = np.linalg.lstsq(basis[:, free] * w[:, None], y * w, rcond=None)
            err = (basis[:, free] @ c - y) * s
            w *= 1.0 + 4.0 * np.abs(err) / np.abs(err).max()
        fixed[top] = float(f16(dict(zip(free, c))[top]))
    return [fixed[k] for k in range(DEG + 1)]


def kernel_eval(s, coef):
    """s times the factor as the kernel forms it: fp16 arithmetic (fused
    multiply-adds rounded once), clamps, then an FP32 product."""
    sh = f16(s)
    with np.errstate(over="ignore"):
        t = f16(sh * sh - 0.5)            # one fused multiply-add
        q = np.full_like(t, coef[DEG])
        for k in range(DEG - 1, -1, -1):
            q = f16(q * t + coef[k])
        factor_h = np.clip(f16(sh * q + 0.5), 0.0, 1.0)
    return np.float32(factor_h) * np.float32(sh), sh


if __name__ == "__main__":
    coef = fit()
    print("coefficients (fp16):", ", ".join(f"{c!r}f16" for c in coef))
    s = np.arange(1 << 16, dtype=np.uint16).view(np.float16).astype(np.float64)
    s = s[np.isfinite(s)]
    g, sh = kernel_eval(s, coef)
    err = np.abs(g - sh * factor(sh))
    print(f"max |s factor - gelu(4 s)/4| in the kernel's arithmetic, every finite fp16 s: {err.max():.2e}")

"""The inference kernel's GELU factor (mlp_infer.h): its fp16 coefficients
are the ones the fit script beside it produces, and evaluated the way the
kernel evaluates them (fp16 fused multiply-adds, t = s^2 - 1/2 unclamped, the
factor clamped to [0, 1], the product in FP32) they stay within 4.7e-4 of
gelu(4 s)/4 in the tanh form for every finite fp16 s, saturating to 0 and s
beyond |s| = 1."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_12471_amd", "csrc")


def _fit_module():
    spec = importlib.util.spec_from_file_location("gelu_poly_fit", os.path.join(CSRC, "gelu_poly_fit.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _kernel_coefficients():
    src = open(os.path.join(CSRC, "mlp_infer.h")).read()
    m = re.search(r"constexpr _Float16 c\[7\] = \{([^}]*)\}", src)
    assert m, "coefficient table not found in mlp_infer.h"
    return [float(x.strip().removesuffix("f16")) for x in m.group(1).split(",")]


def test_kernel_coefficients_are_the_fit():
    G = _fit_module()
    assert _kernel_coefficients() == G.fit()


def test_fp16_evaluation_error_and_saturation():
    G = _fit_module()
    coef = _kernel_coefficients()
    s = np.arange(1 << 16, dtype=np.uint16).view(np.float16).astype(np.float64)
    s = s[np.isfinite(s)]
    g, sh = G.kernel_eval(s, coef)
    exact = sh * G.factor(sh)
    assert np.all(np.isfinite(g))
    assert np.max(np.abs(g - exact)) <= 4.7e-4
    big = sh > 1.0
    np.testing.assert_array_equal(g[big], np.float32(sh[big]))   # factor exactly 1
    assert np.all(np.abs(g[sh < -1.0]) <= 1e-5 * np.abs(sh[sh < -1.0]))

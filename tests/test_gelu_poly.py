"""The forward GEMM epilogue's GELU (a clamped odd polynomial for Phi, in
`csrc/gemm.hip`) against the exact GELU, x Phi(x) with Phi from the error
function, on the CPU.  The constants are read from the kernel source, and the
kernel's sequence of FP32 FMAs is emulated (each FMA rounded once to FP32, the
product of two FP32 values being exact in FP64).  The bounds are the ones the
kernel's comment states."""
import os
import re

import numpy as np
from scipy.special import erf

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2402_18858_amd", "csrc", "gemm.hip")


def _gelu_constants():
    src = open(SRC).read()
    body = src[src.index("float gelu_f(float x) {"):]
    body = body[:body.index("\n}\n")]
    clamp = re.search(r"fmed3f\(x, -([0-9.]+)f, ([0-9.]+)f\)", body)
    centre = re.search(r"fmaf\(xc, xc, -([0-9.]+)f\)", body)
    first = re.search(r"float p = fmaf\(t, ([-0-9.e]+)f, ([-0-9.e]+)f\);", body)
    rest = re.findall(r"p = fmaf\(t, p, ([-0-9.e]+)f\);", body)
    assert clamp and centre and first and rest, "gelu_f no longer has the expected form"
    assert clamp.group(1) == clamp.group(2)
    coef_hi_to_lo = [float(first.group(1)), float(first.group(2))] + [float(c) for c in rest]
    assert "return x * fmaf(xc, p, 0.5f);" in body
    return np.float32(clamp.group(1)), np.float32(centre.group(1)), [np.float32(c) for c in coef_hi_to_lo]


def _fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def _gelu_kernel(x):
    R, s0, coef = _gelu_constants()
    x = np.asarray(x, np.float32)
    xc = np.minimum(np.maximum(x, -R), R)
    t = _fma32(xc, xc, -s0)
    p = _fma32(t, coef[0], coef[1])
    for c in coef[2:]:
        p = _fma32(t, p, c)
    q = _fma32(xc, p, np.float32(0.5))
    phi = q.astype(np.float64)
    return (x * q).astype(np.float32).astype(np.float64), phi


def _gelu_exact(x):
    x = np.asarray(x, np.float64)
    return x * 0.5 * (1.0 + erf(x / np.sqrt(2.0)))


def test_phi_error_on_the_clamped_range():
    x = np.linspace(-4.5, 4.5, 400001).astype(np.float32)
    _, phi = _gelu_kernel(x)
    err = np.abs(phi - 0.5 * (1.0 + erf(x.astype(np.float64) / np.sqrt(2.0))))
    assert err.max() <= 2.2e-7


def test_gelu_absolute_and_relative_error():
    x = np.linspace(-12.0, 12.0, 1200001).astype(np.float32)
    g, _ = _gelu_kernel(x)
    ge = _gelu_exact(x)
    ae = np.abs(g - ge)
    xd = x.astype(np.float64)
    assert ae[np.abs(xd) <= 3.0].max() <= 6.0e-7
    pos = xd > 0.05
    assert (ae[pos] / ge[pos]).max() <= 4.0e-6
    # outside the clamp: x times Phi(+-4.5) (within 3.4e-6 of 1 or 0)
    assert (ae / np.maximum(np.abs(xd), 1.0)).max() <= 4.0e-6


def test_gelu_special_values():
    g, _ = _gelu_kernel(np.array([0.0, np.inf, -np.inf, np.nan], np.float32))
    assert g[0] == 0.0
    assert g[1] == np.inf and g[2] == -np.inf
    assert np.isnan(g[3])

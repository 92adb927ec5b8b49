"""The single-track model's atan on the GPU is an odd polynomial on [0, 1] with the
reflection atan(x) = pi/2 - atan(1/x) beyond.  Its seven float32 coefficients (read here
from the kernel source) are a minimax fit of the absolute error on [0, 1]: the error
alternates in sign at the nine extrema of an equal-ripple curve.  Evaluated in float32 as
the kernel does (Horner with fused multiply-adds), its error against libm's atan stays below
3.5e-7 on [0, 1] and below 4e-7 on the reflected range (float32 rounding of pi/2 - r).
The slip angles' atan takes an odd quintic on [0, 1/4] (three coefficients, a minimax fit
there: 1.2e-7, below 1.5e-7 in float32) and the general atan beyond."""

import math
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2607_25388_amd", "csrc",
                   "sgtp.hip")


def coefficients(start="float atan_poly(float t, float t2)", stop="return p * t;"):
    src = open(SRC).read()
    body = src[src.index(start):]
    body = body[:body.index(stop)]
    return [float.fromhex(h) for h in re.findall(r"(-?0x1\.[0-9a-f]+p[-+]?\d+)f", body)]


def slip_coefficients():
    """The quintic's coefficients, highest degree first (as Horner takes them)."""
    return coefficients("float atan_quintic(float x)", "return p * x;")


def f32(x):
    return np.float32(x)


def fma32(a, b, c):
    # exact product of two float32 values in float64, then one rounding of the sum to float32
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def poly32(t, c):
    t = np.asarray(t, np.float32)
    t2 = (t * t).astype(np.float32)
    p = np.full_like(t, f32(c[0]))
    for k in c[1:]:
        p = fma32(p, t2, f32(k))
    return (p * t).astype(np.float32)


def test_coefficients_are_an_equal_ripple_fit():
    c = coefficients()
    assert len(c) == 7
    t = np.linspace(0.0, 1.0, 20001)
    t2 = t * t
    p = np.full_like(t, c[0])
    for k in c[1:]:
        p = p * t2 + k
    err = p * t - np.arctan(t)
    # local extrema of the error curve (interior) and the end point t = 1
    d = np.diff(err)
    ext = [i + 1 for i in range(len(d) - 1) if d[i] * d[i + 1] < 0] + [len(t) - 1]
    vals = err[ext]
    assert len(vals) >= 8
    assert np.all(np.sign(vals[1:]) != np.sign(vals[:-1])), "the error does not alternate"
    mags = np.abs(vals)
    assert mags.max() < 2.6e-7 and mags.min() > 0.9 * mags.max(), mags


def test_float32_evaluation_error_against_libm():
    c = coefficients()
    rng = np.random.default_rng(1)
    x = np.concatenate([np.linspace(0.0, 1.0, 100001), rng.uniform(0.0, 1.0, 100000)]).astype(np.float32)
    got = poly32(x, c).astype(np.float64)
    ref = np.arctan(x.astype(np.float64))
    assert np.abs(got - ref).max() <= 3.5e-7
    # reflected range |x| > 1: pi/2 - p(1/x) (1/x), the reciprocal rounded to float32
    X = np.concatenate([np.geomspace(1.0, 1e6, 100001), rng.uniform(1.0, 20.0, 100000)]).astype(np.float32)
    r = (np.float32(1.0) / X).astype(np.float32)
    got = (np.float32(1.57079637) - poly32(r, c)).astype(np.float32).astype(np.float64)
    ref = np.arctan(X.astype(np.float64))
    assert np.abs(got - ref).max() <= 4e-7
    # odd: the fast form p(x^2) x is the slow form's copysign(p(|x|^2) |x|, x) bit for bit
    xs = np.linspace(-1.0, 1.0, 20001).astype(np.float32)
    assert np.array_equal(poly32(xs, c), np.copysign(poly32(np.abs(xs), c), xs))


def test_slip_quintic_is_an_equal_ripple_fit_on_a_quarter():
    c = slip_coefficients()
    assert len(c) == 3
    t = np.linspace(0.0, 0.25, 20001)
    t2 = t * t
    p = np.full_like(t, c[0])
    for k in c[1:]:
        p = p * t2 + k
    err = p * t - np.arctan(t)
    d = np.diff(err)
    ext = [i + 1 for i in range(len(d) - 1) if d[i] * d[i + 1] < 0] + [len(t) - 1]
    vals = err[ext]
    assert len(vals) >= 3
    assert np.all(np.sign(vals[1:]) != np.sign(vals[:-1])), "the error does not alternate"
    mags = np.abs(vals)
    assert mags.max() < 1.3e-7 and mags.min() > 0.9 * mags.max(), mags


def test_slip_quintic_float32_error_and_symmetry():
    c = slip_coefficients()
    rng = np.random.default_rng(2)
    x = np.concatenate([np.linspace(0.0, 0.25, 100001), rng.uniform(0.0, 0.25, 100000)]).astype(np.float32)
    got = poly32(x, c).astype(np.float64)
    assert np.abs(got - np.arctan(x.astype(np.float64))).max() <= 1.5e-7
    xs = np.linspace(-0.25, 0.25, 20001).astype(np.float32)
    assert np.array_equal(poly32(xs, c), -poly32(-xs, c))

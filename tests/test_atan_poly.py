"""The slip angle's arctangent in the kernels (atan_mm in
csrc/rollout_step.h): its six coefficients, read from the header, evaluated
the way the kernel does in float32, stay within the stated bound of the true
arctangent on [0, 1] and, through pi/2 - atan(1/|x|), beyond; the sign and
the limits at infinity are right. Host-side check of the product's
constants (no GPU)."""
import os
import re

import numpy as np

from paper_2603_20525_amd import fit_atan

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "paper_2603_20525_amd", "csrc", "rollout_step.h")
BOUND = 4.5e-7  # on [-1, 1]
BOUND_BEYOND = 6e-7  # |x| > 1: the reciprocal (within an ulp on the GPU) and pi/2 - y round too


def header_coefficients():
    src = open(HEADER).read()
    body = src[src.index("float atan_mm(float x)"):]
    body = body[:body.index("return copysignf")]
    vals = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    assert len(vals) == 6, vals
    # the kernel starts Horner from the highest coefficient
    return np.array(vals[::-1], dtype=np.float32)


def kernel_atan(coef, x):
    x = np.asarray(x, dtype=np.float32)
    ax = np.abs(x)
    big = ax > 1
    with np.errstate(divide="ignore"):
        r = np.where(big, (np.float32(1) / ax).astype(np.float32), ax).astype(np.float32)
    y = fit_atan.eval_f32(coef, r)
    y = np.where(big, (np.float32(np.pi / 2) - y).astype(np.float32), y)
    return np.copysign(y, x).astype(np.float32)


def test_header_coefficients_are_the_fit():
    coef, e = fit_atan.fit()
    np.testing.assert_allclose(header_coefficients(), coef, rtol=2e-6, atol=1e-8)
    assert e < 3.2e-7


def test_error_bound_on_the_whole_line():
    coef = header_coefficients()
    x = np.concatenate([np.linspace(0, 1, 200001), 1 / np.linspace(1e-6, 1, 20001),
                        -np.linspace(0, 4, 4001)]).astype(np.float32)
    err = np.abs(kernel_atan(coef, x).astype(np.float64) - np.arctan(x.astype(np.float64)))
    inner = np.abs(x) <= 1
    assert err[inner].max() < BOUND, err[inner].max()
    # beyond 1 the test's reciprocal is correctly rounded; the GPU's is within
    # an ulp of r, which moves atan(r) by at most 6e-8 more
    assert err[~inner].max() + 6e-8 < BOUND_BEYOND, err[~inner].max()


def test_special_values():
    coef = header_coefficients()
    y = kernel_atan(coef, np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan], np.float32))
    assert y[0] == 0 and y[1] == 0 and np.signbit(y[1])
    assert abs(y[2] - np.pi / 4) < BOUND and abs(y[3] + np.pi / 4) < BOUND
    assert y[4] == np.float32(np.pi / 2) and y[5] == -np.float32(np.pi / 2)
    assert np.isnan(y[6])
    # odd symmetry
    x = np.linspace(-3, 3, 601).astype(np.float32)
    np.testing.assert_array_equal(kernel_atan(coef, x), -kernel_atan(coef, -x))

"""Error bounds of the march's shortcut forms of softplus and opacity.

The march kernel takes softplus(x) = log(1 + e^x) in Goldberg's form
log(u) e / (u - 1), u = 1 + e, and the opacity 1 - e^-s in Kahan's form
(1 - u) s / -log(u), u = e^-s, near s = 0 (the density activation and the
per-sample alpha of the compositing, Sec. II-B).  Its logarithm is the
hardware log2 times ln 2 rounded to float, and its e^x the hardware exp2 of
x log2(e) with the product's rounding error applied as a first-order
correction.  These tests
emulate those float32 steps in numpy, with exp2, log2 and the reciprocal
correctly rounded, and check the relative error bounds quoted for the kernel
against float64 references.  They exercise the arithmetic of the forms, not
the kernel itself; the GPU parity tests compare the kernel's images with the
oracle.
"""
import numpy as np
import pytest

F = np.float32
LOG2E_HI = F(1.44269502162933349609375)      # log2(e) rounded to float
LOG2E_LO = F(1.925963033500011079e-8)        # log2(e) - LOG2E_HI
LN2 = F(0.693147182)                         # ln 2 rounded to float


def rn(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma(a, b, c):
    # a * b is exact in float64 for float32 operands; one rounding to float32
    return rn(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def exp2_cr(x):
    return rn(np.exp2(x.astype(np.float64)))


def log2_cr(x):
    with np.errstate(divide="ignore", invalid="ignore"):
        return rn(np.log2(x.astype(np.float64)))


def rcp_cr(x):
    with np.errstate(divide="ignore"):
        return rn(1.0 / x.astype(np.float64))


def exp_hw(x):
    hi = rn(x * LOG2E_HI)
    lo = fma(x, LOG2E_LO, fma(x, LOG2E_HI, -hi))
    eh = exp2_cr(hi)
    return fma(eh, rn(lo * LN2), eh)


def ln_hw(u):
    return rn(log2_cr(u) * LN2)


def softplus_march(x):
    big = x > F(15)
    e = exp_hw(np.where(big, -x, x).astype(np.float32))
    u = rn(F(1) + e)
    with np.errstate(invalid="ignore"):
        l = np.where(u == F(1), e, rn(ln_hw(u) * rn(e * rcp_cr(rn(u - F(1))))))
    return np.where(big, rn(x + e), l)


def opacity_march(s):
    u = exp2_cr(rn(s * F(-1.44269504088896341)))
    with np.errstate(invalid="ignore"):
        k = np.where(u == F(1), s, rn(rn(rn(F(1) - u) * s) * rcp_cr(-ln_hw(u))))
    return np.where(u > F(0.5), k, rn(F(1) - u))


@pytest.fixture(scope="module")
def rng():
    return np.random.default_rng(20240418)


def test_exp_hw_relative_error(rng):
    x = np.concatenate([rng.uniform(-80, 15, 400_000), np.linspace(-1, 1, 100_001)]).astype(np.float32)
    ref = np.exp(x.astype(np.float64))
    rel = np.abs(exp_hw(x) - ref) / ref
    assert rel.max() < 1.3e-7, rel.max()
    # the plain product x log2(e) alone loses up to |x| log2(e) ulp of the
    # exponent's fraction: the correction is what keeps the bound
    plain = exp2_cr(rn(x * LOG2E_HI))
    assert (np.abs(plain - ref) / ref).max() > 4e-7


def test_softplus_relative_error(rng):
    x = np.concatenate([rng.uniform(-30, 25, 600_000), rng.uniform(-1e-3, 1e-3, 100_000),
                        np.linspace(-40, 20, 200_001), np.float32([0.0, 15.0, 15.000001, -15.0])]).astype(np.float32)
    ref = np.log1p(np.exp(x.astype(np.float64)))
    rel = np.abs(softplus_march(x) - ref) / ref
    assert rel.max() < 3.2e-7, (rel.max(), x[np.argmax(rel)])


def test_softplus_form_beats_direct_log(rng):
    # log(1 + e) taken directly loses every digit of e below the rounding of
    # 1 + e; Goldberg's form keeps them (the reason the march uses it)
    x = rng.uniform(-30, -10, 100_000).astype(np.float32)
    ref = np.log1p(np.exp(x.astype(np.float64)))
    direct = ln_hw(rn(F(1) + exp_hw(x)))
    assert (np.abs(direct - ref) / ref).max() > 1e-2
    assert (np.abs(softplus_march(x) - ref) / ref).max() < 3.2e-7


def test_opacity_relative_error(rng):
    s = np.concatenate([rng.uniform(0, 1e-3, 300_000), rng.uniform(0, 12, 300_000),
                        np.logspace(-9, 1, 200_000), np.float32([1e-30, np.log(2.0), 20.0])]).astype(np.float32)
    ref = -np.expm1(-s.astype(np.float64))
    rel = np.abs(opacity_march(s) - ref) / ref
    assert rel.max() < 2.5e-7, (rel.max(), s[np.argmax(rel)])
    # 1 - e^-s taken directly cancels near s = 0
    direct = rn(F(1) - exp2_cr(rn(s * F(-1.44269504088896341))))
    small = s < 1e-4
    assert (np.abs(direct[small] - ref[small]) / ref[small]).max() > 1e-2

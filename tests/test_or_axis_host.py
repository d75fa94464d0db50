"""Accuracy of the over-relaxation axis of the fixed-point path (no GPU).

The fixed-point over-relaxation reflects a 16-bit angle about the local field,
theta' = 2 phi_q - theta, where phi_q is atan2(h_y, h_x) on the 2^16 grid
(Sec. 3, improved equilibrium dynamics; the reflection is then accepted by a
Metropolis test).  The device evaluates atan on [0, 1] by an odd polynomial.
Its coefficients are read from the device source, the polynomial is evaluated
in FP32 with one rounding per fused multiply-add, and the error must stay below
the bound the source states (an eighth of the angle quantum), so that 2 phi_q
is off the exact rounding by at most one grid step.
"""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1211_3991_amd", "csrc", "fix16_common.hpp")


def _coefficients():
    body = open(SRC).read()
    body = body[body.index("uint32_t field_axis2("):]
    body = body[:body.index("float a = p * t;")]
    first = re.search(r"float p = ([-0-9.e]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, t2, ([-0-9.e]+)f\);", body)
    return [np.float32(float(v)) for v in [first] + rest]       # highest degree first


def _fma32(a, b, c):
    # a*b is exact in FP64 for FP32 operands; the sum is rounded to FP64 and then to FP32
    return (a.astype(np.float64) * b.astype(np.float64) + np.float64(c)).astype(np.float32)


def _atan01(t):
    t = t.astype(np.float32)
    t2 = (t * t).astype(np.float32)
    c = _coefficients()
    p = np.full_like(t, c[0])
    for ck in c[1:]:
        p = _fma32(p, t2, ck)
    return (p * t).astype(np.float32)


def test_polynomial_within_stated_bound():
    t = np.linspace(0.0, 1.0, 1 << 20)
    err = np.abs(_atan01(t).astype(np.float64) - np.arctan(t.astype(np.float32).astype(np.float64)))
    assert len(_coefficients()) == 5                      # degree 9
    assert err.max() < 1.3e-5, err.max()
    assert 1.3e-5 < (2 * np.pi / 65536) / 7               # under an eighth of the quantum (with margin)


def _axis2(hx, hy):
    """The device's 2 phi on the 2^16 grid: a = atan(min/max) by the
    polynomial, signed by the XOR of the sign bits of hx, hy and |hx| - |hy|,
    scaled by 2^16 / pi and rounded, plus a half turn when |hy| > |hx|."""
    ax, ay = np.abs(hx), np.abs(hy)
    mx, mn = np.maximum(np.maximum(ax, ay), np.float32(1e-30)), np.minimum(ax, ay)
    a = _atan01((mn / mx).astype(np.float32)).astype(np.float64)
    d = (ax - ay).astype(np.float32)
    neg = np.signbit(hx) ^ np.signbit(hy) ^ np.signbit(d)
    a = np.where(neg, -a, a)
    return (np.rint(a * 65536 / np.pi).astype(np.int64) + np.where(d < 0, 32768, 0)) & 0xFFFF


def _axis2_exact(hx, hy):
    return np.rint(np.arctan2(hy.astype(np.float64), hx.astype(np.float64)) * 65536 / np.pi).astype(np.int64) & 0xFFFF


def test_axis_within_one_grid_step():
    """2 phi on the 2^16 grid, with the octant restored as on the device, is
    the exact rounding or one step from it over random fields (about 15% of
    them one step off: the reflected angle is then one quantum from the
    exact reflection, which the Metropolis test of the move absorbs)."""
    rng = np.random.default_rng(7)
    hx, hy = (rng.standard_normal(200000) * 3).astype(np.float32), (rng.standard_normal(200000) * 3).astype(np.float32)
    d = (_axis2(hx, hy) - _axis2_exact(hx, hy)) & 0xFFFF
    d = np.minimum(d, 65536 - d)
    assert d.max() <= 1 and d.mean() < 0.25, (d.max(), d.mean())


def test_axis_octants_and_degenerate_fields():
    """Every octant, the axes with either sign of zero, the diagonals and the
    zero field: the doubled angle is the exact one within a grid step, and a
    zero field gives the axis 0 (a reflection theta -> -theta)."""
    ang = np.arange(16) * (np.pi / 8) + 0.1                         # interior points of all octants
    hx = np.concatenate([np.cos(ang), [1, -1, 0, 0, -0.0, 1, -1, 1, -1], [0.0, -0.0]]).astype(np.float32)
    hy = np.concatenate([np.sin(ang), [0, 0, 1, -1, 1, -0.0, -0.0, 1, -1], [0.0, -0.0]]).astype(np.float32)
    got, exact = _axis2(hx, hy), _axis2_exact(hx, hy)
    d = (got - exact) & 0xFFFF
    assert np.minimum(d, 65536 - d).max() <= 1, (got, exact)
    assert got[-1] == 0 and got[-2] == 0


def _const(name):
    body = open(SRC).read()
    return float(re.search(r"constexpr float %s = ([-0-9.e]+)f;" % name, body).group(1))


def test_axis_error_bound_used_by_the_sure_accept_test():
    """The doubled axis differs from twice the field's angle by under
    7.44e-5 rad (the polynomial's error twice over plus half a grid step), the
    bound the over-relaxation's sure-accept test takes for |dE| / |h|; and the
    test's constants clear the inequality it rests on."""
    rng = np.random.default_rng(11)
    hx = (rng.standard_normal(400000) * 3).astype(np.float32)
    hy = (rng.standard_normal(400000) * 3).astype(np.float32)
    got = _axis2(hx, hy) * (2 * np.pi / 65536)
    exact = 2 * np.arctan2(hy.astype(np.float64), hx.astype(np.float64))
    d = np.angle(np.exp(1j * (got - exact)))
    assert np.abs(d).max() < 7.44e-5, np.abs(d).max()
    trig, exp2 = _const("kTrigErr"), _const("kExp2Err")
    delta_e = 7.44e-5 + 2 * trig + 4e-7
    assert _const("kOrSureCoef") > 65536 * np.log(2) * delta_e * 1.1
    assert 65534 + 65536 * exp2 + 0.01 < 65535


def test_sure_accept_bound_against_worst_case_full_test():
    """Random fields, angles, temperatures and uniforms, with fields up to
    |h_x| + |h_y| = 60 and beta up to 10, near the bound: whenever the
    sure-accept test passes, the full acceptance test accepts even with every
    error at its worst (the (cos, sin) values off by kTrigErr against the
    move, 2^x low by kExp2Err, and the FP32 rounding of dE against it)."""
    rng = np.random.default_rng(3)
    n = 1_000_000
    scale = rng.uniform(0.0, 20.0, n).astype(np.float32)
    hx = (rng.standard_normal(n) * scale).astype(np.float32)
    hy = (rng.standard_normal(n) * scale).astype(np.float32)
    th = rng.integers(0, 65536, n)
    beta = rng.uniform(0.05, 10.0, n)
    factor = (-beta.astype(np.float32) * np.float32(1.4426950408889634)).astype(np.float32)
    h1 = (np.abs(hx) + np.abs(hy)).astype(np.float32)
    coef = np.float32(-_const("kOrSureCoef")) * factor
    # uniforms at and just below the sure-accept threshold, where it is tightest
    u = np.clip(np.floor(65534.0 - coef.astype(np.float64) * h1 - rng.uniform(0, 3, n)), 0, 65535)
    sure = (coef.astype(np.float64) * h1 + u) <= 65534.0
    new = (_axis2(hx, hy) - th) & 0xFFFF
    a0, a1 = th * (2 * np.pi / 65536), new * (2 * np.pi / 65536)
    de = hx.astype(np.float64) * (np.cos(a0) - np.cos(a1)) + hy.astype(np.float64) * (np.sin(a0) - np.sin(a1))
    worst = de + h1 * (2 * _const("kTrigErr") + 4e-7)                  # every error against the move
    p = np.exp2(-np.maximum(worst, 0.0) * beta * 1.4426950408889634) * (1 - _const("kExp2Err"))
    q = p * 65536 - u
    assert sure.mean() > 0.5
    assert np.all(q[sure] >= 1.0), (q[sure].min(), np.argmin(q[sure]))
    # and the bound is of the right size: |dE| / |h| comes within a factor 2.5 of 7.44e-5 on these fields
    hn = np.sqrt(hx.astype(np.float64) ** 2 + hy.astype(np.float64) ** 2)
    assert (np.abs(de) / np.maximum(hn, 1e-30)).max() > 0.4 * 7.44e-5

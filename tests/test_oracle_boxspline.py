"""Pins of the oracle's box-spline evaluator (Sec. III-A, eq. (9), (16), (18)).

The oracle evaluates the 3-direction box spline as a moving average (eq. (9))
of the closed-form 2-direction spline.  These tests pin it to the paper's
truncated-power formula (eq. (18): forward differences of (x)_+^2 / 2!),
evaluated here in exact rational arithmetic, and to properties any box spline
must have: unit mass, symmetry, support, partition of unity.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate


def exact_box(x, widths):
    """Centred unit-mass box spline by eq. (16)/(18), exact rationals.

    With n non-zero directions w the non-centred spline is
    Delta_w1 ... Delta_wn (y)_+^(n-1) / (n-1)!, divided by prod |w_i| (each
    elementary box has height 1/|w|); centring shifts y by sum(w)/2.  Zero
    directions are dropped (Sec. IV-A: a delta distribution)."""
    w = [Fraction(abs(float(t))) for t in widths if float(t) != 0.0]
    x = Fraction(float(x))
    n = len(w)
    if n == 1:
        return float(Fraction(1) / w[0]) if abs(x) < w[0] / 2 else 0.0
    fact = 1
    for k in range(2, n):
        fact *= k
    total = Fraction(0)
    for bits in range(1 << n):
        sign = 1
        y = x
        for i in range(n):
            s = -1 if (bits >> i) & 1 else 1
            sign *= s
            y += s * w[i] / 2
        if y > 0:
            total += sign * y ** (n - 1)
    den = Fraction(fact)
    for t in w:
        den *= t
    return float(total / den)


def _cases(rng, count):
    out = []
    for _ in range(count):
        kind = rng.integers(0, 6)
        w = rng.uniform(0.05, 2.0, 3)
        if kind == 1:      # one tiny width (near axis-aligned ray)
            w[rng.integers(0, 3)] = 10.0 ** rng.uniform(-17, -6)
        elif kind == 2:    # one zero width (axis-aligned ray)
            w[rng.integers(0, 3)] = 0.0
        elif kind == 3:    # c = a + b exactly (breakpoints coincide)
            w[2] = w[0] + w[1]
        elif kind == 4:    # equal widths
            w[1] = w[0]
        support = 0.5 * w.sum()
        x = rng.uniform(-1.1, 1.1) * support
        out.append((x, *w))
    return out


def test_box3_matches_exact_truncated_power(oracle_mod):
    rng = np.random.default_rng(123)
    worst = 0.0
    for x, a, b, c in _cases(rng, 3000):
        got = oracle_mod.box3(x, a, b, c)
        ref = exact_box(x, (a, b, c))
        scale = 1.0 / max(a, b, c)        # the spline's maximum is <= 1/max width
        worst = max(worst, abs(got - ref) / scale)
    assert worst < 1e-14, worst


def test_box3_special_points(oracle_mod):
    # three equal widths: the quadratic B-spline, value 3/4 at its centre
    assert oracle_mod.box3(0.0, 1.0, 1.0, 1.0) == pytest.approx(0.75, abs=1e-15)
    assert oracle_mod.box3(0.5, 1.0, 1.0, 1.0) == pytest.approx(0.5, abs=1e-15)
    assert oracle_mod.box3(1.5, 1.0, 1.0, 1.0) == 0.0
    # two vanishing widths leave a box of height 1/c
    assert oracle_mod.box3(0.2, 0.0, 0.0, 0.8) == pytest.approx(1.25, abs=1e-15)
    assert oracle_mod.box3(0.41, 0.0, 0.0, 0.8) == 0.0
    # c >= a + b: the plateau equals 1/c
    assert oracle_mod.box3(0.05, 0.1, 0.2, 1.0) == pytest.approx(1.0, abs=1e-15)


def test_box2_matches_exact(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(2000):
        a, b = rng.uniform(0.0, 2.0, 2)
        if rng.random() < 0.2:
            a = 0.0
        x = rng.uniform(-1.2, 1.2) * 0.5 * (a + b)
        got = oracle_mod.box2(x, a, b)
        ref = exact_box(x, (a, b))
        assert abs(got - ref) <= 1e-14 / max(a, b), (x, a, b, got, ref)


@pytest.mark.parametrize("w", [(0.3, 0.7, 1.1), (1e-9, 0.7, 0.9), (0.0, 0.5, 0.5), (0.4, 0.4, 2.0)])
def test_box3_unit_mass_symmetry_support(oracle_mod, w):
    half = 0.5 * sum(w)
    f = lambda t: oracle_mod.box3(t, *w)
    pts = sorted({0.5 * abs(s1 * w[0] + s2 * w[1] + s3 * w[2])
                  for s1 in (-1, 1) for s2 in (-1, 1) for s3 in (-1, 1)})
    mass = 2.0 * integrate.quad(f, 0.0, half, points=pts[:-1] or None, limit=200,
                                epsabs=1e-14, epsrel=1e-14)[0]
    assert mass == pytest.approx(1.0, abs=1e-10)
    for t in np.linspace(0.0, 1.2 * half, 57):
        assert f(t) == pytest.approx(f(-t), abs=1e-15)
    assert f(half) == 0.0 and f(half * 1.0001) == 0.0
    assert f(half * 0.999) > 0.0


@pytest.mark.parametrize("a,b,tau", [(0.3, 0.9, 1.0), (0.01, 0.99, 0.5), (0.7, 0.7, 1.5)])
def test_box3_partition_of_unity(oracle_mod, a, b, tau):
    """Shifts of M_[a, b, tau] by multiples of tau, times tau, sum to one: the
    detector cells tile the line and the blur has unit mass (Theorem 1)."""
    for x in np.linspace(-0.6, 0.6, 37):
        total = sum(tau * oracle_mod.box3(x - m * tau, a, b, tau) for m in range(-10, 11))
        assert total == pytest.approx(1.0, abs=1e-14)

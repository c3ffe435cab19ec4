"""Exact geometric quantities written from first principles, for pinning the
oracle.  Nothing here uses box splines: chords come from clipping a line
against a square, areas from clipping a polygon, and the reference projector
(Sec. V, "Ref") integrates exact chords across a detector cell.
"""
from __future__ import annotations

import math

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def fan_frame(theta, dsc, dsd):
    u = np.array([math.cos(theta), math.sin(theta)])
    e = np.array([math.sin(theta), -math.cos(theta)])
    p = dsc * u
    return u, e, p


def detector_point(theta, dsc, dsd, s):
    u, e, p = fan_frame(theta, dsc, dsd)
    return p - dsd * u + s * e


def line_chord(p, d, lo, hi):
    """Length of the line p + t d (|d| = 1, all t) inside the box [lo, hi]."""
    t0, t1 = -math.inf, math.inf
    for ax in range(2):
        if d[ax] == 0.0:
            if not (lo[ax] <= p[ax] <= hi[ax]):
                return 0.0
            continue
        ta = (lo[ax] - p[ax]) / d[ax]
        tb = (hi[ax] - p[ax]) / d[ax]
        t0 = max(t0, min(ta, tb))
        t1 = min(t1, max(ta, tb))
    return max(0.0, t1 - t0)


def pixel_box(i, j, nx, ny, pixel):
    kx = (i - 0.5 * (nx - 1)) * pixel
    ky = (j - 0.5 * (ny - 1)) * pixel
    return np.array([kx - 0.5 * pixel, ky - 0.5 * pixel]), np.array([kx + 0.5 * pixel, ky + 0.5 * pixel])


def fan_chord(theta, dsc, dsd, s, lo, hi):
    """Exact length of the fan ray through detector coordinate s inside a box."""
    u, e, p = fan_frame(theta, dsc, dsd)
    q = p - dsd * u + s * e
    d = (q - p) / np.linalg.norm(q - p)
    return line_chord(p, d, lo, hi)


def corner_shadows(theta, dsc, dsd, lo, hi):
    u, e, p = fan_frame(theta, dsc, dsd)
    out = []
    for x in (lo[0], hi[0]):
        for y in (lo[1], hi[1]):
            c = np.array([x, y])
            out.append(dsd * (e @ c) / (dsc - u @ c))
    return out


def ref_entry(theta, dsc, dsd, s_m, tau, lo, hi):
    """Reference projector: (1/tau) * integral over the cell of the exact chord
    (unit-mass detector blur, detector coordinate).  Composite 24-point
    Gauss-Legendre between the cell edges and the corner shadows, where the
    chord is smooth."""
    a, b = s_m - 0.5 * tau, s_m + 0.5 * tau
    cuts = sorted([a, b] + [c for c in corner_shadows(theta, dsc, dsd, lo, hi) if a < c < b])
    total = 0.0
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        if x1 <= x0:
            continue
        xs = 0.5 * (x1 - x0) * _GL_X + 0.5 * (x1 + x0)
        f = [fan_chord(theta, dsc, dsd, s, lo, hi) for s in xs]
        total += 0.5 * (x1 - x0) * float(np.dot(_GL_W, f))
    return total / tau


def clip_halfplane(poly, n, c):
    """Sutherland-Hodgman: keep the part of `poly` with n . x <= c."""
    out = []
    k = len(poly)
    for idx in range(k):
        P, Q = poly[idx], poly[(idx + 1) % k]
        fp, fq = n @ P - c, n @ Q - c
        if fp <= 0:
            out.append(P)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append(P + t * (Q - P))
    return out


def polygon_area(poly):
    """Gauss's (shoelace) area formula, eq. (8)."""
    if len(poly) < 3:
        return 0.0
    P = np.array(poly)
    x, y = P[:, 0], P[:, 1]
    return 0.5 * abs(float(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1))))


def strip_pixel_area(e, s_lo, s_hi, lo, hi):
    """Area of {x : s_lo <= e . x <= s_hi} intersected with the box [lo, hi]."""
    poly = [np.array([lo[0], lo[1]]), np.array([hi[0], lo[1]]),
            np.array([hi[0], hi[1]]), np.array([lo[0], hi[1]])]
    poly = clip_halfplane(poly, e, s_hi)
    if poly:
        poly = clip_halfplane(poly, -e, -s_lo)
    return polygon_area(poly)


def disk_fan_projection(theta, dsc, dsd, s_m, tau, radius):
    """Bin-averaged fan-beam line integral of the centred unit disk: the chord
    2 sqrt(r^2 - d^2)_+ with d = dsc |sin(atan(s/dsd))| the distance of the ray
    from the centre, averaged over the cell (Gauss-Legendre, split at the
    tangent rays)."""
    a, b = s_m - 0.5 * tau, s_m + 0.5 * tau
    # tangent rays: d = r  <=>  s = +-dsd r / sqrt(dsc^2 - r^2)
    st = dsd * radius / math.sqrt(dsc * dsc - radius * radius)
    cuts = sorted([a, b] + [c for c in (-st, st) if a < c < b])
    total = 0.0
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        xs = 0.5 * (x1 - x0) * _GL_X + 0.5 * (x1 + x0)
        d = dsc * np.abs(xs) / np.sqrt(dsd * dsd + xs * xs)
        f = 2.0 * np.sqrt(np.maximum(radius * radius - d * d, 0.0))
        total += 0.5 * (x1 - x0) * float(np.dot(_GL_W, f))
    return total / tau


# ---- arc detector: cells on the circle of radius dsd around the source; the
# detector coordinate s is arc length, so the ray of s leaves the central ray
# (towards -u) at the angle s / dsd ----

def arc_direction(theta, dsc, dsd, s):
    u, e, p = fan_frame(theta, dsc, dsd)
    g = s / dsd
    return -math.cos(g) * u + math.sin(g) * e


def arc_chord(theta, dsc, dsd, s, lo, hi):
    """Exact length of the arc-detector ray through coordinate s inside a box."""
    u, e, p = fan_frame(theta, dsc, dsd)
    return line_chord(p, arc_direction(theta, dsc, dsd, s), lo, hi)


def arc_corner_shadows(theta, dsc, dsd, lo, hi):
    """Arc coordinates of the rays through the four corners of a box."""
    u, e, p = fan_frame(theta, dsc, dsd)
    out = []
    for x in (lo[0], hi[0]):
        for y in (lo[1], hi[1]):
            c = np.array([x, y])
            out.append(dsd * math.atan2(e @ c, dsc - u @ c))
    return out


def ref_entry_arc(theta, dsc, dsd, s_m, tau, lo, hi):
    """Reference projector of the arc detector: (1/tau) * integral over the
    cell's arc of the exact chord, split at the corner rays."""
    a, b = s_m - 0.5 * tau, s_m + 0.5 * tau
    cuts = sorted([a, b] + [c for c in arc_corner_shadows(theta, dsc, dsd, lo, hi) if a < c < b])
    total = 0.0
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        if x1 <= x0:
            continue
        xs = 0.5 * (x1 - x0) * _GL_X + 0.5 * (x1 + x0)
        f = [arc_chord(theta, dsc, dsd, s, lo, hi) for s in xs]
        total += 0.5 * (x1 - x0) * float(np.dot(_GL_W, f))
    return total / tau


def disk_arc_projection(dsc, dsd, s_m, tau, radius):
    """Cell-averaged line integral of the centred unit disk on the arc
    detector: the ray at angle s / dsd passes at dsc |sin(s / dsd)| from the
    centre; split at the tangent rays."""
    a, b = s_m - 0.5 * tau, s_m + 0.5 * tau
    st = dsd * math.asin(radius / dsc)
    cuts = sorted([a, b] + [c for c in (-st, st) if a < c < b])
    total = 0.0
    for x0, x1 in zip(cuts[:-1], cuts[1:]):
        xs = 0.5 * (x1 - x0) * _GL_X + 0.5 * (x1 + x0)
        d = dsc * np.abs(np.sin(xs / dsd))
        f = 2.0 * np.sqrt(np.maximum(radius * radius - d * d, 0.0))
        total += 0.5 * (x1 - x0) * float(np.dot(_GL_W, f))
    return total / tau

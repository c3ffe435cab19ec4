"""Pins of the oracle's geometry variants: the arc detector and a cell pitch
different from the cell width.

Arc detector (the derivation applied to cells on a circle around the source):
* tau -> 0: the entry equals the exact chord of the arc ray (eq. (16) exact);
* the frame quantities equal their polar forms: s' = rho sin(g_k - g_m) and
  tau' = L * 2 tan(tau / (2 D_sd)), rho and g_k the distance and angle of the
  pixel centre seen from the source;
* the model approaches the exact blurred projection (chord averaged over the
  cell's arc) as in the flat case, closer as the source moves away;
* a uniform disk projects to its closed-form cell average;
* adjoint identity, pruned == dense, non-zero count.

Pitch != width (parallel beam, where the model is exact, Theorem 1):
* the entry equals area(strip of the cell's width inside the pixel) / tau;
* when the width is an integer multiple of the pitch, the cells' boxes tile
  the line, so sum_m pitch * A_(m,k) = delta^2 exactly.
"""
import math

import numpy as np
import pytest

import exact_geometry as eg
from paper_1907_10526_amd import phantoms


def _arc(oracle_mod, n, dsc, dsd, angs, nd, tau, pixel=1.0, spacing=None):
    return oracle_mod.Geometry(n, n, pixel, dsc, dsd, angs, nd, tau, det_spacing=spacing,
                               mode=oracle_mod.FAN_ARC)


def test_arc_zero_blur_entry_is_exact_chord(oracle_mod):
    n, dsc, dsd, nd, spacing = 12, 40.0, 80.0, 64, 0.7
    rng = np.random.default_rng(3)
    angs = np.concatenate([[0.0, math.pi / 2, math.pi / 4, math.pi], rng.uniform(0, 2 * math.pi, 6)])
    g = _arc(oracle_mod, n, dsc, dsd, angs, nd, 0.0, spacing=spacing)
    worst, hits = 0.0, 0
    for v, th in enumerate(angs):
        for i in range(n):
            for j in range(n):
                lo, hi = eg.pixel_box(i, j, n, n, 1.0)
                for m in range(nd):
                    s = (m - 0.5 * (nd - 1)) * spacing
                    ch = eg.arc_chord(th, dsc, dsd, s, lo, hi)
                    worst = max(worst, abs(ch - g.entry(v, m, i, j)))
                    hits += ch > 0
    assert hits > 2000
    assert worst < 1e-12, worst


def test_arc_frame_matches_polar_form(oracle_mod):
    n, dsc, dsd, nd, tau = 16, 30.0, 55.0, 40, 0.9
    angs = np.array([0.0, 0.7, 2.2, 4.0])
    g = _arc(oracle_mod, n, dsc, dsd, angs, nd, tau)
    worst = 0.0
    for v, th in enumerate(angs):
        u = np.array([math.cos(th), math.sin(th)])
        e = np.array([math.sin(th), -math.cos(th)])
        for i, j in [(0, 0), (15, 3), (7, 8), (2, 14)]:
            k = np.array([(i - 7.5), (j - 7.5)])
            rho = float(np.linalg.norm(k - dsc * u))
            gk = math.atan2(e @ k, dsc - u @ k)
            for m in (0, 7, 19, 20, 39):
                gm = (m - 0.5 * (nd - 1)) * tau / dsd
                sp, z1, z2, tp, L = g.entry_terms(v, m, i, j)
                worst = max(worst, abs(sp - rho * math.sin(gk - gm)),
                            abs(L - rho * math.cos(gk - gm)),
                            abs(tp - L * 2.0 * math.tan(0.5 * tau / dsd)))
                # projected pixel widths: delta |w_perp|, w_perp the ray normal
                wp = math.cos(gm) * e + math.sin(gm) * u
                worst = max(worst, abs(abs(z1) - abs(wp[0])), abs(abs(z2) - abs(wp[1])))
    assert worst < 1e-12, worst


def _arc_ref_error(oracle_mod, n, dsc, dsd, tau, angs, pixels, pad=8):
    nd = 2 * int(math.ceil(0.75 * n * dsd / dsc / tau)) + pad
    g = _arc(oracle_mod, n, dsc, dsd, angs, nd, tau)
    worst = 0.0
    for v, th in enumerate(angs):
        for i, j in pixels:
            lo, hi = eg.pixel_box(i, j, n, n, 1.0)
            for m in range(nd):
                s = (m - 0.5 * (nd - 1)) * tau
                r = eg.ref_entry_arc(th, dsc, dsd, s, tau, lo, hi)
                e = g.entry(v, m, i, j)
                if r == 0.0 and e == 0.0:
                    continue
                worst = max(worst, abs(r - e))
    return worst


def test_arc_cnsf_close_to_reference_projector(oracle_mod):
    angs = np.linspace(0.0, 2 * math.pi, 13)[:-1] + 0.05
    pix = [(0, 0), (7, 7), (3, 5), (7, 0)]
    e_small = _arc_ref_error(oracle_mod, 8, 128.0, 256.0, 1.5, angs, pix)
    e_mid = _arc_ref_error(oracle_mod, 8, 200.0, 400.0, 0.5, angs, pix)
    e_far = _arc_ref_error(oracle_mod, 8, 1000.0, 1500.0, 1.0, angs, pix)
    assert e_small < 1e-3, e_small
    assert e_far < e_mid < e_small, (e_small, e_mid, e_far)
    assert e_far < 2e-4


def test_arc_disk_projection_closed_form(oracle_mod):
    n, dsc, dsd, nd, tau = 64, 128.0, 256.0, 128, 1.5
    angs = 2 * math.pi * np.arange(12) / 90
    ref = np.array([[eg.disk_arc_projection(dsc, dsd, (m - 0.5 * (nd - 1)) * tau, tau, 24.0)
                     for m in range(nd)] for _ in angs])
    g = _arc(oracle_mod, n, dsc, dsd, angs, nd, tau)
    err = np.linalg.norm(g.forward(phantoms.disk(n, 24.0, 1.0).astype(np.float64)) - ref) / np.linalg.norm(ref)
    g2 = _arc(oracle_mod, 2 * n, dsc, dsd, angs, nd, tau, pixel=0.5)
    y2 = g2.forward(phantoms.disk(2 * n, 48.0, 0.5).astype(np.float64))
    err2 = np.linalg.norm(y2 - ref) / np.linalg.norm(ref)
    assert err < 1e-2, err
    assert err2 < 0.4 * err, (err, err2)


def test_arc_adjoint_pruning_and_count(oracle_mod):
    n, nd = 16, 48
    rng = np.random.default_rng(9)
    angs = np.concatenate([[0.0, math.pi / 2, math.pi / 4], rng.uniform(0, 2 * math.pi, 9)])
    g = _arc(oracle_mod, n, 14.0, 40.0, angs, nd, 1.3, spacing=1.1)
    c = phantoms.uniform((n, n), 41).astype(np.float64)
    y = phantoms.uniform((len(angs), nd), 42).astype(np.float64)
    f, b = g.forward(c), g.back(y)
    assert np.array_equal(f, g.forward(c, dense=True))
    assert np.array_equal(b, g.back(y, dense=True))
    lhs, rhs = float(np.sum(f * y)), float(np.sum(c * b))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    dense = sum(g.entry(v, m, i, j) != 0.0 for v in range(len(angs)) for m in range(nd)
                for i in range(n) for j in range(n))
    assert g.count_nonzero() == dense


def test_arc_and_flat_agree_on_the_central_ray(oracle_mod):
    """The central cell's ray is the same line for both detectors and its
    blur agrees to second order in tau / D_sd."""
    n, dsc, dsd, nd, tau = 16, 60.0, 120.0, 41, 1.0
    angs = np.array([0.3, 1.9])
    ga = _arc(oracle_mod, n, dsc, dsd, angs, nd, tau)
    gf = oracle_mod.Geometry(n, n, 1.0, dsc, dsd, angs, nd, tau)
    m = nd // 2
    for v in range(2):
        for i in range(n):
            for j in range(n):
                ta, tf = ga.entry_terms(v, m, i, j), gf.entry_terms(v, m, i, j)
                assert ta[0] == pytest.approx(tf[0], abs=1e-12)
                assert ta[3] == pytest.approx(tf[3], rel=(tau / dsd) ** 2)


@pytest.mark.parametrize("spacing,width", [(0.5, 0.8), (1.0, 0.6), (0.7, 1.4)])
def test_parallel_pitch_differs_from_width_strip_area(oracle_mod, spacing, width):
    n, nd = 8, 36
    rng = np.random.default_rng(2)
    angs = np.concatenate([[0.0, math.pi / 4, math.pi / 2], rng.uniform(0, 2 * math.pi, 4)])
    g = oracle_mod.Geometry(n, n, 1.0, 50.0, 100.0, angs, nd, width, det_spacing=spacing,
                            mode=oracle_mod.PARALLEL)
    worst = 0.0
    for v, th in enumerate(angs):
        e = np.array([math.sin(th), -math.cos(th)])
        for i in range(n):
            for j in range(n):
                lo, hi = eg.pixel_box(i, j, n, n, 1.0)
                for m in range(nd):
                    s = (m - 0.5 * (nd - 1)) * spacing
                    ref = eg.strip_pixel_area(e, s - 0.5 * width, s + 0.5 * width, lo, hi) / width
                    worst = max(worst, abs(ref - g.entry(v, m, i, j)))
    assert worst < 1e-13, worst


@pytest.mark.parametrize("ratio", [2, 3])
def test_parallel_integer_width_ratio_tiles_mass(oracle_mod, ratio):
    n, nd, spacing, pix = 8, 80, 0.35, 1.2
    angs = np.linspace(0.0, math.pi, 9)
    g = oracle_mod.Geometry(n, n, pix, 50.0, 100.0, angs, nd, ratio * spacing, det_spacing=spacing,
                            mode=oracle_mod.PARALLEL)
    for v in range(len(angs)):
        for i, j in [(0, 0), (3, 4), (7, 2)]:
            tot = sum(spacing * g.entry(v, m, i, j) for m in range(nd))
            assert tot == pytest.approx(pix * pix, abs=1e-13)

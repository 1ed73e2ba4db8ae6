"""Pins for the oracle's PQ (Sec. 4.1, Eq. 1-2) and LOD weights (Sec. 4.2.1, Eq. 3)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import pq
from oracle.encoding import level_star, lod_weights

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_pq_unit_peak_is_exactly_one():
    # rational identity of Eq. 2: (c1 + c2) / (1 + c3) = 2520/2520
    assert pq.pq_encode(1.0) == pytest.approx(1.0, abs=1e-15)
    assert (pq.C1 + pq.C2) == pytest.approx(1.0 + pq.C3, abs=1e-15)


def test_pq_zero_is_c1_pow_m2():
    assert pq.pq_encode(0.0) == pytest.approx((107 / 128) ** (2523 / 32), rel=1e-12)
    assert 7.2e-7 < pq.pq_encode(0.0) < 7.4e-7


def test_pq_published_reference_points():
    g = json.load(open(os.path.join(GOLD, "pq_st2084_points.json")))
    for p in g["points"]:
        e = pq.pq_encode(p["nits"] / 10000.0)
        assert abs(e - p["pq"]) <= g["tolerance_pq"], p
        assert int(round(float(e) * 1023)) == p["code10"], p


def test_pq_linear_one_is_100_nits():
    # Sec. 4.1: linear color 1 maps to 100 cd/m^2
    assert pq.linear_to_pq(1.0) == pytest.approx(pq.pq_encode(0.01), rel=1e-15)
    assert pq.pq_to_linear(pq.linear_to_pq(1.0)) == pytest.approx(1.0, rel=1e-12)


def test_pq_round_trip_and_monotone():
    y = np.concatenate([[0.0], np.logspace(-9, 0, 2000)])
    e = pq.pq_encode(y)
    assert np.all(np.diff(e) > 0)
    back = pq.pq_decode(e)
    assert np.max(np.abs(back - y) / np.maximum(y, 1e-7)) < 1e-9
    assert np.all((e >= 0) & (e <= 1))


def test_lod_weight_tables():
    g = json.load(open(os.path.join(GOLD, "lod_weights.json")))
    for c in g["cases"]:
        w = lod_weights(np.array([c["L_star"]]), 8)[0]
        np.testing.assert_allclose(w, c["w"], atol=1e-12)


def test_lod_weights_continuous_and_monotone():
    ls = np.linspace(0, 7.999, 4001)
    w = lod_weights(ls, 8)
    assert np.all(np.diff(w, axis=1) <= 1e-12)      # non-increasing in level
    assert np.max(np.abs(np.diff(w, axis=0))) < 2 * (ls[1] - ls[0]) + 1e-12  # continuous in L*
    for n in range(1, 7):                              # across integers
        a, b = lod_weights(np.array([n - 1e-9, n + 1e-9]), 8)
        assert np.max(np.abs(a - b)) < 1e-8


def test_nyquist_level_matches_voxel_size():
    # Sec. 4.2.1: level L has voxel size (s f^L)^-1; a footprint of half that
    # voxel gives L* = L exactly (features twice the footprint are resolvable).
    field = {"extent": 1.0, "base_res": 128.0, "growth": 1.4, "lod_bias": 0.0}
    s, f = np.float64(np.float32(128.0)), np.float64(np.float32(1.4))
    for L in range(16):
        rhat = 0.5 / (s * f ** L)
        assert level_star(np.array([1.0]), np.array([rhat]), field)[0] == pytest.approx(L, abs=1e-9)


def test_lod_bias_shifts_level_exactly_and_clamps():
    base = {"extent": 2.0, "base_res": 16.0, "growth": 1.5, "lod_bias": 0.0}
    t, r = np.array([0.7, 3.0]), np.array([1e-3, 1e-3])
    l0 = level_star(t, r, base)
    for b in (-2.0, -0.5, 1.0, 3.0):
        lb = level_star(t, r, dict(base, lod_bias=b))
        np.testing.assert_allclose(lb, np.maximum(l0 + b, 0.0), atol=1e-12)
    # a huge footprint clamps to L* = 0: level 0 keeps weight 1
    far = level_star(np.array([1e6]), np.array([1.0]), base)
    assert far[0] == 0.0 and lod_weights(far, 4)[0].tolist() == [1, 0, 0, 0]
    # L* doubles footprint -> drops exactly one "octave" of log_f 2 levels
    l2 = level_star(2 * t, r, base)
    np.testing.assert_allclose(l0 - l2, math.log(2) / math.log(np.float32(1.5)), atol=1e-9)


def test_srgb_transfer_reference_points_and_tonemap():
    g = json.load(open(os.path.join(GOLD, "srgb_points.json")))
    for lin, enc in g["points"]:
        assert abs(float(pq.srgb_oetf(lin)) - enc) <= g["tolerance"], (lin, enc)
    v = np.linspace(0, 1, 10001)
    s = pq.srgb_oetf(v)
    assert np.all(np.diff(s) > 0)
    # exposure: +1 EV doubles the linear value before the curve; clipping above 1
    e = pq.linear_to_pq(np.array([0.1, 0.3, 2.0]))
    np.testing.assert_allclose(pq.pq_to_display(e, 1.0), pq.srgb_oetf(2 * np.array([0.1, 0.3, 2.0])), atol=1e-12)
    assert abs(pq.pq_to_display(e, 0.0)[2] - 1.0) < 1e-12

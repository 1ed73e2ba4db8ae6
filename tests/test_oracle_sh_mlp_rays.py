"""Pins for the oracle's SH basis, MLPs and canonical rays / cone pitch."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre

from oracle import mlp as M
from oracle.rays import canonical_rays, cone_pitch, fp64_directions
from oracle.sh import sh_basis

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_sh_axis_closed_forms():
    k0 = 1 / (2 * math.sqrt(math.pi))
    k1 = math.sqrt(3 / (4 * math.pi))
    axes = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], float)
    Y = sh_basis(axes, 2)
    np.testing.assert_allclose(Y[:, 0], k0, atol=1e-15)
    # band 1 ordered m = -1, 0, 1  ->  (y, z, x) times sqrt(3 / 4 pi)
    np.testing.assert_allclose(Y[:, 1:4], k1 * axes[:, [1, 2, 0]], atol=1e-15)
    # band 2 at +z: only m = 0 survives, (1/4) sqrt(5/pi) (3 z^2 - 1) = (1/2) sqrt(5/pi)
    Y2 = sh_basis(np.array([[0, 0, 1.0]]), 3)[0, 4:9]
    np.testing.assert_allclose(Y2, [0, 0, 0.5 * math.sqrt(5 / math.pi), 0, 0], atol=1e-15)


def _quadrature(n):
    z, wz = roots_legendre(n)
    phi = (np.arange(2 * n) + 0.5) * (2 * math.pi / (2 * n))
    Z, P = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(wz[:, None], 2 * n, 1) * (2 * math.pi / (2 * n))
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3)
    return d, W.reshape(-1)


def test_sh_orthonormal_by_quadrature():
    d, w = _quadrature(24)
    Y = sh_basis(d, 5)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(25), atol=1e-12)


def test_sh_addition_theorem_against_scipy_legendre():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((50, 3))
    b = rng.standard_normal((50, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = sh_basis(a, 5), sh_basis(b, 5)
    cos = np.sum(a * b, 1)
    for l in range(5):
        sl = slice(l * l, (l + 1) * (l + 1))
        lhs = np.sum(Ya[:, sl] * Yb[:, sl], 1)
        rhs = (2 * l + 1) / (4 * math.pi) * eval_legendre(l, cos)
        np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_mlp_hand_example():
    g = json.load(open(os.path.join(GOLD, "mlp_hand_example.json")))
    m = {k: np.array(v, float) for k, v in g["mlp"].items()}
    sigma, geo = M.density_mlp(np.array([g["feats"]]), m)
    assert sigma[0] == pytest.approx(g["sigma"], abs=1e-15)
    np.testing.assert_allclose(geo[0], g["geo"], atol=1e-15)
    rgb = M.color_mlp(geo, np.array([g["sh"]]), m)
    np.testing.assert_allclose(rgb[0], g["rgb"], atol=1e-15)


def test_mlp_zero_weights_closed_form():
    rng = np.random.default_rng(2)
    m = {"W1": np.zeros((32, 64)), "b1": rng.normal(size=64), "W2": np.zeros((64, 16)),
         "b2": rng.normal(size=16), "W3": np.zeros((31, 64)), "b3": rng.normal(size=64),
         "W4": np.zeros((64, 64)), "b4": rng.normal(size=64), "W5": np.zeros((64, 3)),
         "b5": rng.normal(size=3)}
    sigma, geo = M.density_mlp(rng.normal(size=(10, 32)), m)
    np.testing.assert_allclose(sigma, math.exp(m["b2"][0]), rtol=1e-15)
    np.testing.assert_allclose(geo, np.tile(m["b2"][1:], (10, 1)), atol=0)
    rgb = M.color_mlp(geo, rng.normal(size=(10, 16)), m)
    np.testing.assert_allclose(rgb, np.tile(1 / (1 + np.exp(-m["b5"])), (10, 1)), rtol=1e-15)


def _cam(R, pos, W=64, fov=60.0):
    fx = (W / 2) / math.tan(math.radians(fov) / 2)
    return {"c2w": np.concatenate([R, np.array(pos)[:, None]], 1).astype(np.float32),
            "fx": np.float32(fx), "fy": np.float32(fx), "cx": np.float32(W / 2), "cy": np.float32(W / 2)}


def test_rays_axes_and_symmetry():
    cam = _cam(np.eye(3), [0.1, 0.2, 0.3], W=64)
    # principal point between pixels 31 and 32: the two central rays mirror in x
    o, d = canonical_rays(cam, np.array([31, 32, 0, 63]), np.array([31, 31, 10, 10]))
    assert d[0, 0] == -d[1, 0] and d[0, 1] == d[1, 1] and d[0, 2] == d[1, 2]
    assert d[2, 0] == -d[3, 0] and d[2, 1] == d[3, 1]
    assert np.all(o == np.array([0.1, 0.2, 0.3], np.float32))
    # FP32 canonical directions are within a few ulps of the exact ones
    i, j = np.meshgrid(np.arange(64), np.arange(64))
    _, d32 = canonical_rays(cam, i.ravel(), j.ravel())
    d64 = fp64_directions(cam, i.ravel(), j.ravel())
    assert np.max(np.abs(d32 - d64)) < 4 * 2.0 ** -24
    assert d32.dtype == np.float32


def test_cone_pitch_closed_form_at_centre():
    fx = 800.0
    cam = {"c2w": np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32),
           "fx": np.float32(fx), "fy": np.float32(fx), "cx": np.float32(100.5), "cy": np.float32(50.5)}
    # pixel 100 has a = 0; its right neighbour a = 1/fx: angle atan(1/fx)
    r = cone_pitch(cam, np.array([100]), np.array([50]))[0]
    assert r == pytest.approx(2 * math.sin(math.atan(1 / fx) / 2), rel=1e-12)
    assert cone_pitch(cam, np.array([100]), np.array([50]), scale=0.5)[0] == pytest.approx(r / 2, rel=1e-15)

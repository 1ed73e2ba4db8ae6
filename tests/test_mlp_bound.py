"""The a-priori 16-bit MLP error bound (tests/mlp_bound.py) holds for an
emulation of the 16-bit arithmetic on the CPU: operands rounded to nearest
FP16 / BF16, products and sums in FP32.  The GPU parity test of the 16-bit
MLP stage uses that bound as its per-sample tolerance."""
import numpy as np
import pytest

from mlp_bound import mlp16_bounds, mlp16_rgb_rms_bound
from oracle.mlp import color_mlp, density_mlp
from oracle.sh import sh_basis
from paper_2311_02542_amd import synth


def _round16(x, compute):
    x = np.asarray(x, np.float32)
    if compute == "f16":
        return x.astype(np.float16).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16           # nearest even in the top 16 bits
    return r.astype(np.uint32).view(np.float32)


def _layer16(W, b, x, compute):
    xr = _round16(x, compute).astype(np.float64)
    Wr = _round16(W, compute).astype(np.float64)
    # exact products accumulated in FP32, one term at a time
    acc = np.zeros((x.shape[0], W.shape[1]), np.float32)
    for i in range(W.shape[0]):
        acc = (acc + (xr[:, i:i + 1] * Wr[i:i + 1, :]).astype(np.float32)).astype(np.float32)
    return (acc + np.asarray(b, np.float32)).astype(np.float32)


def _emulate(feats, sh, mlp, compute):
    m = {k: np.asarray(v, np.float32) for k, v in mlp.items()}
    h = np.maximum(_layer16(m["W1"], m["b1"], feats, compute), 0)
    o = _layer16(m["W2"], m["b2"], h, compute)
    z = np.concatenate([o[:, 1:], sh.astype(np.float32)], axis=1)
    c1 = np.maximum(_layer16(m["W3"], m["b3"], z, compute), 0)
    c2 = np.maximum(_layer16(m["W4"], m["b4"], c1, compute), 0)
    lg = _layer16(m["W5"], m["b5"], c2, compute).astype(np.float64)
    return np.exp(o[:, 0].astype(np.float64)), 1 / (1 + np.exp(-lg))


@pytest.mark.parametrize("compute", ["f16", "bf16"])
@pytest.mark.parametrize("case", ["blobs64", "room256"])
def test_bound_contains_emulated_16bit_mlp(case, compute):
    f = synth.field_blobs64() if case == "blobs64" else synth.field_room256()
    L = int(f["n_levels"])
    rng = np.random.default_rng(5)
    n = 2000
    feats = rng.uniform(-0.1, 0.1, (n, 2 * L)).astype(np.float32)
    d = rng.standard_normal((n, 3))
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    sh = sh_basis(d, int(f["sh_bands"]))
    s_ref, geo = density_mlp(feats.astype(np.float64), f["mlp"])
    c_ref = color_mlp(geo, sh, f["mlp"])
    s_tol, c_worst = mlp16_bounds(feats, sh, f["mlp"], compute)
    c_tol = mlp16_rgb_rms_bound(feats, sh, f["mlp"], compute)
    s_em, c_em = _emulate(feats, sh, f["mlp"], compute)
    s_err = np.abs(s_em / s_ref - 1)
    c_err = np.abs(c_em - c_ref)
    assert (s_err <= s_tol).all(), f"sigma: {np.max(s_err / s_tol):.3g} of the bound"
    assert (c_err <= c_worst).all()
    assert (c_err <= c_tol).all(), f"rgb: {np.max(c_err / c_tol):.3g} of the 6-sigma tolerance"
    # the sigma bound is a worst case, but not a vacuous one; the color
    # tolerance is far inside the worst case
    assert np.median(s_tol) < (0.02 if compute == "f16" else 0.15)
    assert np.median(c_tol) < 0.05 * np.median(c_worst)
    print(f"{case} {compute}: sigma err/bound max {np.max(s_err / s_tol):.3f}, "
          f"median bound {np.median(s_tol):.2e}; rgb err/bound max {np.max(c_err / c_tol):.3f}, "
          f"median bound {np.median(c_tol):.2e}")

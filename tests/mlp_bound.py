"""A-priori bound on the per-sample error of the 16-bit MLP path (FP16 or
BF16 MFMA operands, FP32 accumulation), derived from its arithmetic rather
than measured.  Test infrastructure (not collected by pytest).

Model of the arithmetic, layer by layer (Sec. 6 MLPs):
* every operand an MFMA reads -- encoded features, SH values, weights,
  hidden activations, the geometry outputs fed to the color MLP -- is the
  exact value plus the error it already carries, rounded to nearest in the
  element type: relative error at most u (2^-11 FP16, 2^-8 BF16) plus, for
  FP16, half its subnormal spacing (2^-25) in absolute terms;
* products of 16-bit operands are exact in FP32; the accumulation over n
  terms and the bias addition are FP32, with error at most (n + 2) 2^-24
  times the sum of absolute values;
* ReLU is 1-Lipschitz, so errors pass through it unchanged.
The bound is carried in FP64 from the exact activations of the plain
definition.  sigma = exp(o0) then has relative error at most exp(E0) - 1,
and the sigmoid (slope at most 1/4) turns a logit error E into at most E/4.

That worst case adds |W| times the incoming error at every layer, which over
the three 64-wide color layers is a thousand times what rounding produces.
For colors the statistical model of the same arithmetic is used instead:
each rounding is an independent error, uniform within +-u of the value
(variance u^2 x^2 / 3), variances add through the products and the FP32
sums, and the tolerance is six standard deviations of the logit error.
"""
import numpy as np

U16 = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
TINY16 = {"f16": 2.0 ** -25, "bf16": 0.0}
U32 = 2.0 ** -24


def _w(mlp, k):
    return np.asarray(mlp[k], np.float64)


def _layer(W, b, x, e_in, u, tiny):
    """Exact pre-activation y = x W + b and a bound on the 16-bit path's
    error in it, for inputs carrying absolute error e_in before rounding."""
    e_op = e_in + u * (np.abs(x) + e_in) + tiny           # operand after rounding
    x_hat = np.abs(x) + e_op                              # bound on |operand|
    aW = np.abs(W)
    prod = x_hat @ (u * aW + tiny) + e_op @ aW            # |w^ x^ - w x| summed
    n = W.shape[0]
    acc = (n + 2) * U32 * (x_hat @ ((1 + u) * aW + tiny) + np.abs(b))
    return x @ W + b, prod + acc


def mlp16_bounds(feats, sh, mlp, compute):
    """Per-sample bounds (sigma relative error, RGB absolute error) of the
    16-bit path for features [n, 2L] and SH values [n, nsh] given exactly
    (the test feeds them as FP32 inputs; the GPU evaluates SH in FP32)."""
    u, tiny = U16[compute], TINY16[compute]
    f = np.asarray(feats, np.float64)
    y1, e1 = _layer(_w(mlp, "W1"), _w(mlp, "b1"), f, np.zeros_like(f), u, tiny)
    h1 = np.maximum(y1, 0.0)
    o, e2 = _layer(_w(mlp, "W2"), _w(mlp, "b2"), h1, e1, u, tiny)
    sh = np.asarray(sh, np.float64)
    z = np.concatenate([o[:, 1:], sh], axis=1)
    ez = np.concatenate([e2[:, 1:], 16 * U32 * (np.abs(sh) + 1.0)], axis=1)   # FP32 SH polynomials
    y3, e3 = _layer(_w(mlp, "W3"), _w(mlp, "b3"), z, ez, u, tiny)
    y4, e4 = _layer(_w(mlp, "W4"), _w(mlp, "b4"), np.maximum(y3, 0.0), e3, u, tiny)
    _, e5 = _layer(_w(mlp, "W5"), _w(mlp, "b5"), np.maximum(y4, 0.0), e4, u, tiny)
    # exp and sigmoid in FP32 add a few ulp on top
    sig_rel = np.expm1(e2[:, 0]) + 8 * U32
    rgb_abs = e5 / 4.0 + 1e-6
    return sig_rel, rgb_abs


def _layer_var(W, b, x, v_in, u):
    """Exact y = x W + b and the variance of the 16-bit path's error in it
    under independent, zero-mean roundings."""
    v_op = v_in + (u * u / 3.0) * (x * x + v_in)
    W2 = W * W
    v = v_op @ W2 + (x * x) @ ((u * u / 3.0) * W2)
    v += W.shape[0] * (U32 * U32 / 3.0) * ((x * x) @ W2 + b * b)
    return x @ W + b, v


def mlp16_rgb_rms_bound(feats, sh, mlp, compute, k=6.0):
    """k standard deviations of the 16-bit path's RGB error per sample and
    channel, under the statistical model (module docstring)."""
    u = U16[compute]
    f = np.asarray(feats, np.float64)
    y1, v1 = _layer_var(_w(mlp, "W1"), _w(mlp, "b1"), f, np.zeros_like(f), u)
    o, v2 = _layer_var(_w(mlp, "W2"), _w(mlp, "b2"), np.maximum(y1, 0.0), v1, u)
    sh = np.asarray(sh, np.float64)
    z = np.concatenate([o[:, 1:], sh], axis=1)
    vz = np.concatenate([v2[:, 1:], (16 * U32) ** 2 * (sh * sh + 1.0)], axis=1)
    y3, v3 = _layer_var(_w(mlp, "W3"), _w(mlp, "b3"), z, vz, u)
    y4, v4 = _layer_var(_w(mlp, "W4"), _w(mlp, "b4"), np.maximum(y3, 0.0), v3, u)
    _, v5 = _layer_var(_w(mlp, "W5"), _w(mlp, "b5"), np.maximum(y4, 0.0), v4, u)
    return k * np.sqrt(v5) / 4.0 + 1e-6

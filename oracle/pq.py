"""PQ (SMPTE ST 2084) perceptual quantiser, FP64 -- Sec. 4.1, Eq. 1-2.

The paper maps a luminance in [0, 10000] cd/m^2 to the unit range with
PQ(Y) = ((c1 + c2 Y^m1) / (1 + c3 Y^m1))^m2 and maps a linear color value of
1 to 100 cd/m^2.  Reading: the formula takes Y normalised by 10000 (only
then does PQ(1 normalised) = 1), applied per RGB channel.
"""
import numpy as np

M1 = 1305.0 / 8192.0
M2 = 2523.0 / 32.0
C1 = 107.0 / 128.0
C2 = 2413.0 / 128.0
C3 = 2392.0 / 128.0
PEAK_NITS = 10000.0
NITS_PER_LINEAR_UNIT = 100.0


def pq_encode(y_norm):
    """Eq. 1 on a luminance normalised by 10000 cd/m^2 (y_norm in [0, 1])."""
    y = np.asarray(y_norm, np.float64)
    ym = np.power(np.maximum(y, 0.0), M1)
    return np.power((C1 + C2 * ym) / (1.0 + C3 * ym), M2)


def pq_decode(e):
    """Algebraic inverse of Eq. 1: normalised luminance from a PQ value."""
    e = np.asarray(e, np.float64)
    ep = np.power(np.maximum(e, 0.0), 1.0 / M2)
    return np.power(np.maximum(ep - C1, 0.0) / (C2 - C3 * ep), 1.0 / M1)


def linear_to_pq(lin):
    """Linear HDR color (1.0 = 100 cd/m^2, Sec. 4.1) to PQ units."""
    return pq_encode(np.asarray(lin, np.float64) * (NITS_PER_LINEAR_UNIT / PEAK_NITS))


def pq_to_linear(e):
    """PQ units back to linear HDR color (Sec. 4.1 scale)."""
    return pq_decode(e) * (PEAK_NITS / NITS_PER_LINEAR_UNIT)


def srgb_oetf(v):
    """sRGB transfer function (IEC 61966-2-1) on linear values in [0, 1]
    (display output, reading R33)."""
    v = np.clip(np.asarray(v, np.float64), 0.0, 1.0)
    return np.where(v <= 0.0031308, 12.92 * v, 1.055 * np.power(v, 1.0 / 2.4) - 0.055)


def pq_to_display(e, exposure_ev=0.0):
    """Display tonemap of a PQ color (Sec. 4.1, Fig. exposure-swipe): decode to
    linear HDR, scale by 2^EV, clip to [0, 1], apply the sRGB transfer.
    Reading: the paper sweeps exposure at render time without giving its
    tonemapper; a clipped exposure scale with the sRGB curve is the plain one."""
    return srgb_oetf(pq_to_linear(e) * (2.0 ** exposure_ev))

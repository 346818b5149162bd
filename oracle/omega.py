"""The random sketch matrix Omega (paper, Section 3: Omega has i.i.d. N(0,1)
entries; Algorithm 1 draws it once).  TEST INFRASTRUCTURE (see package doc).

The paper does not say how Omega is drawn.  Both this oracle and the GPU
library draw it from the same published definition, implemented twice:

* uniform bits: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11), key = (seed, stream), counter =
  (c, 0, 0, 0).  Counter c yields four 64-bit words w0..w3;
* uniforms: u1 = ((w0 >> 11) + 1) * 2^-53 in (0, 1],
            u2 = (w1 >> 11) * 2^-53       in [0, 1)   (same for w2, w3);
* normals (Box-Muller): rho = sqrt(-2 ln u1),
            z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2);
* Omega (l x n, row-major) entry (i, j) has flat index q = i*n + j and is
  normal number (q mod 4) of counter c = q // 4, stream 1.

ln, cos and sin are evaluated with the fixed sequence of IEEE double
operations written below (exact range reduction plus a truncated series,
every operation rounded on its own), so that any IEEE-754 implementation that
performs the same operations in the same order produces the same bits.
"""

import numpy as np

STREAM_OMEGA = 1

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)
# Philox4x64 round multipliers and key increments (the SC'11 paper, Table 2 /
# its reference implementation)
_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)


def _mulhilo64(a, m):
    """(hi, lo) 64-bit halves of the 128-bit product a*m (a array, m scalar)."""
    lo = a * m
    a_lo, a_hi = a & _M32, a >> _S32
    m_lo, m_hi = m & _M32, m >> _S32
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.

    ctr: uint64 array of shape (..., 4); key: two uint64 values.
    Returns uint64 array of shape (..., 4).
    """
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.array(ctr[..., i], dtype=np.uint64) for i in range(4))
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        for _ in range(10):
            hi0, lo0 = _mulhilo64(x0, _PHILOX_M0)
            hi1, lo1 = _mulhilo64(x2, _PHILOX_M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = np.uint64((int(k0) + int(_PHILOX_W0)) & 0xFFFFFFFFFFFFFFFF)
            k1 = np.uint64((int(k1) + int(_PHILOX_W1)) & 0xFFFFFFFFFFFFFFFF)
        return np.stack([x0, x1, x2, x3], axis=-1)


# ---- elementary functions from + - * / sqrt only -------------------------

_LN2_HI = 6.93147180369123816490e-01   # ln 2 rounded to 32 significant bits
_LN2_LO = 1.90821492927058770002e-10   # ln 2 - _LN2_HI
_SQRT_HALF = 0.70710678118654752440
_HALF_PI = 1.57079632679489661923


def ln(x):
    """Natural log of x > 0.

    x = m * 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) with
    s = (m - 1)/(m + 1), |s| < 0.172, summed as 2 s (1 + s^2/3 + ... +
    s^20/21) by Horner; ln x = e*LN2_HI + (ln m + e*LN2_LO).
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # m in [0.5, 1)
    low = m < _SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    acc = 1.0 / 21.0
    for k in range(9, -1, -1):              # coefficients 1/19, 1/17, ..., 1/1
        acc = acc * z + 1.0 / (2 * k + 1)
    lnm = (2.0 * s) * acc
    return e * _LN2_HI + (lnm + e * _LN2_LO)


def _sin_poly(t):
    """sin t for 0 <= t <= pi/4: t (1 - t^2/3! + ... - t^18/19!) by Horner."""
    z = t * t
    acc = -1.0 / 121645100408832000.0           # -1/19!
    fact = [1.0, 6.0, 120.0, 5040.0, 362880.0, 39916800.0, 6227020800.0,
            1307674368000.0, 355687428096000.0]  # (2k+1)!, k = 0..8
    for k in range(8, -1, -1):
        c = 1.0 / fact[k]
        if k % 2:
            c = -c
        acc = acc * z + c
    return t * acc


def _cos_poly(t):
    """cos t for 0 <= t <= pi/4: 1 - t^2/2! + ... + t^20/20! by Horner."""
    z = t * t
    acc = 1.0 / 2432902008176640000.0            # 1/20!
    fact = [1.0, 2.0, 24.0, 720.0, 40320.0, 3628800.0, 479001600.0,
            87178291200.0, 20922789888000.0, 6402373705728000.0]  # (2k)!, k = 0..9
    for k in range(9, -1, -1):
        c = 1.0 / fact[k]
        if k % 2:
            c = -c
        acc = acc * z + c
    return acc


def cos_sin_2pi(u):
    """(cos 2 pi u, sin 2 pi u) for u in [0, 1).

    Quadrant q = floor(4u), g = 4u - q (both exact).  For g <= 1/2 the angle
    inside the quadrant is t = (pi/2) g; otherwise t = (pi/2)(1 - g) and the
    roles of sin and cos swap.  The quadrant then rotates (c, s).
    """
    u = np.asarray(u, dtype=np.float64)
    f = u * 4.0
    q = np.floor(f)
    g = f - q
    upper = g > 0.5
    t = np.where(upper, _HALF_PI * (1.0 - g), _HALF_PI * g)
    st = _sin_poly(t)
    ct = _cos_poly(t)
    c1 = np.where(upper, st, ct)   # cos of (pi/2) g
    s1 = np.where(upper, ct, st)   # sin of (pi/2) g
    qi = q.astype(np.int64) & 3
    c = np.choose(qi, [c1, -s1, -c1, s1])
    s = np.choose(qi, [s1, c1, -s1, -c1])
    return c, s


def gaussians(seed, stream, count):
    """The first ``count`` normal numbers of (seed, stream)."""
    nctr = (count + 3) // 4
    ctr = np.zeros((nctr, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nctr, dtype=np.uint64)
    key = (int(seed) & 0xFFFFFFFFFFFFFFFF, stream)
    w = philox4x64_10(ctr, key)
    scale = 2.0 ** -53
    z = np.empty((nctr, 4))
    for a, b in ((0, 1), (2, 3)):
        u1 = ((w[:, a] >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * scale
        u2 = (w[:, b] >> np.uint64(11)).astype(np.float64) * scale
        rho = np.sqrt(-2.0 * ln(u1))
        c, s = cos_sin_2pi(u2)
        z[:, a] = rho * c
        z[:, b] = rho * s
    return z.reshape(-1)[:count]


def omega(seed, l, n, stream=STREAM_OMEGA):
    """Omega in R^{l x n}, i.i.d. N(0,1), as defined in the module docstring;
    ``stream`` > 1 gives the fresh sketching matrices of Algorithm 2 (the
    j-th recomputation draws from stream 1 + j)."""
    if l * n == 0:
        return np.zeros((l, n))
    return gaussians(seed, stream, l * n).reshape(l, n)

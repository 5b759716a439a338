"""Kaiser-Bessel window (oracle; test infrastructure only).

The paper leaves the window open (Remark 2.1) and names Kaiser-Bessel as the window of its
inner NFFTs (Example 3.13, Example 3.21).  Reading used throughout (stated once here):

  shape parameter  b = pi (2 - 1/sigma)
  window, in grid units v = M_sigma x:
      w(v) = sinh(b sqrt(m^2 - v^2)) / (pi sqrt(m^2 - v^2))      for |v| <= m
           (limit b/pi where the square root vanishes)
  truncation w_m = chi_[-m/M_sigma, m/M_sigma] * w   (Section 2.1, closed interval)
  Fourier transform of the untruncated window, as Section 2.1 requires for the entries of D:
      w_hat(k) = (1/M_sigma) I_0(m sqrt(b^2 - (2 pi k / M_sigma)^2))
  so the deconvolution factor (2.4) is 1/(M_sigma w_hat(k)) = 1/I_0(...).

I_0 is summed from its power series sum_n (z^2/4)^n / (n!)^2 until the terms stop changing the
float64 sum (all terms are positive, so there is no cancellation).
"""
from __future__ import annotations

import numpy as np


def shape_b(sigma: float) -> float:
    return np.pi * (2.0 - 1.0 / sigma)


def i0_series(z) -> np.ndarray:
    """Modified Bessel function I_0 by its power series, float64."""
    z = np.asarray(z, dtype=np.float64)
    q = (z * 0.5) ** 2
    term = np.ones_like(z)
    total = np.ones_like(z)
    n = 1
    while True:
        term = term * q / float(n * n)
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
        n += 1
        if n > 2000:
            raise RuntimeError("I0 series did not converge")
    return total


def window(v, m: int, b: float) -> np.ndarray:
    """Truncated window w_m in grid units v = M_sigma x (zero for |v| > m)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    inside = np.abs(v) <= m
    t2 = (m - v[inside]) * (m + v[inside])
    t = np.sqrt(t2)
    val = np.empty_like(t)
    pos = t > 0
    val[pos] = np.sinh(b * t[pos]) / (np.pi * t[pos])
    val[~pos] = b / np.pi
    out[inside] = val
    return out


def window_deriv(v, m: int, b: float) -> np.ndarray:
    """d w / d v of the truncated window inside its support (the jump at |v| = m is not
    included).  w(v) = sinh(b t)/(pi t), t = sqrt(m^2 - v^2):
        dw/dv = -v (b t cosh(b t) - sinh(b t)) / (pi t^3),
    with the series (x cosh x - sinh x)/x^3 = sum_{n>=1} 2n x^(2n-2)/(2n+1)! for small b t."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    inside = np.abs(v) <= m
    vv = v[inside]
    t = np.sqrt((m - vv) * (m + vv))
    x = b * t
    ratio = np.empty_like(t)  # (x cosh x - sinh x)/x^3
    small = x < 1e-2
    xs = x[small]
    # 1/3 + x^2/30 + x^4/840 + x^6/45360
    ratio[small] = 1.0 / 3 + xs ** 2 / 30 + xs ** 4 / 840 + xs ** 6 / 45360
    xl = x[~small]
    ratio[~small] = (xl * np.cosh(xl) - np.sinh(xl)) / xl ** 3
    out[inside] = -vv * b ** 3 * ratio / np.pi
    return out


def window_hat(k, Ms: int, m: int, b: float) -> np.ndarray:
    """Fourier transform w_hat(k) of the (untruncated) window, cf. (2.3)."""
    k = np.asarray(k, dtype=np.float64)
    arg = b * b - (2 * np.pi * k / Ms) ** 2
    if np.any(arg < 0):
        raise ValueError("frequency beyond the window's main lobe (sigma < 1?)")
    return i0_series(m * np.sqrt(arg)) / Ms


def deconv(k, Ms: int, m: int, b: float) -> np.ndarray:
    """Diagonal entries of D in (2.4): 1 / (M_sigma w_hat(k))."""
    return 1.0 / (Ms * window_hat(k, Ms, m, b))

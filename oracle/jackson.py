"""Jackson-Chebyshev approximation of the ideal low-pass (oracle; test only).

Eq. (1) defines the ideal low-pass h_lc(lambda) = 1 for lambda <= lc, 0 above,
on [0, 2].  Sec. 4.3 approximates it by a Chebyshev polynomial of order p
whose coefficients carry Jackson damping factors (after Napoli, Polizzi and
Saad), which suppress the Gibbs oscillation around the cut-off.  The paper does
not print the formulas; written out on x = lambda - 1 in [-1, 1]:

* Chebyshev coefficients of the step 1[x <= xc], xc = lc - 1, theta_c = arccos(xc):
      c_0 = 1 - theta_c / pi,   c_m = -2 sin(m theta_c) / (m pi)   (m >= 1);
  these are (1/pi) int h(x) / sqrt(1 - x^2) dx for m = 0 and
  (2/pi) int h(x) T_m(x) / sqrt(1 - x^2) dx for m >= 1;
* Jackson factors for p + 1 terms, alpha = pi / (p + 2):
      g_m = [(p + 2 - m) cos(m alpha) + sin(m alpha) cot(alpha)] / (p + 2);
* h~(lambda) = sum_{m=0}^{p} g_m c_m T_m(lambda - 1).
"""
from __future__ import annotations

import numpy as np


def cheb_step_coeffs(lc: float, p: int) -> np.ndarray:
    """Undamped Chebyshev coefficients c_0..c_p of 1[lambda <= lc] on [0, 2]."""
    xc = min(max(lc - 1.0, -1.0), 1.0)
    th = np.arccos(xc)
    m = np.arange(1, p + 1, dtype=np.float64)
    c = np.empty(p + 1)
    c[0] = 1.0 - th / np.pi
    c[1:] = -2.0 * np.sin(m * th) / (m * np.pi)
    return c


def jackson_factors(p: int) -> np.ndarray:
    """Jackson damping factors g_0..g_p."""
    a = np.pi / (p + 2)
    m = np.arange(p + 1, dtype=np.float64)
    return ((p + 2 - m) * np.cos(m * a) + np.sin(m * a) / np.tan(a)) / (p + 2)


def lowpass_coeffs(lc: float, p: int, damping: bool = True) -> np.ndarray:
    """Coefficients a_m of h~_lc in the basis T_m(lambda - 1), m = 0..p."""
    c = cheb_step_coeffs(lc, p)
    return c * jackson_factors(p) if damping else c


def evaluate(a: np.ndarray, lam) -> np.ndarray:
    """sum_m a_m T_m(lambda - 1) with T_m(cos t) = cos(m t)."""
    lam = np.asarray(lam, dtype=np.float64)
    t = np.arccos(np.clip(lam - 1.0, -1.0, 1.0))
    m = np.arange(len(a), dtype=np.float64)
    return np.cos(np.multiply.outer(t, m)) @ a

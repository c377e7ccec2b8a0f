"""Zolotarev's optimal rational approximation of x^(-1/2) on [eps, 1].

The rational approximation of the heavy-sector determinant (Section 4.2, the
partial fractions solved by the multishift CG) uses the best uniform relative
approximation of x^(-1/2) by a rational function of degree (n, n).  Zolotarev
gave it in closed form through Jacobi elliptic functions: with the
complementary modulus k' = sqrt(1 - eps) and K' = K(k'),

    R(x) = d * prod_{l=1..n} (x + eps c_{2l}) / (x + eps c_{2l-1}),
    c_m  = sn^2(m K' / (2n+1); k') / (1 - sn^2(m K' / (2n+1); k'))

(the c_m belong to the interval scaled to [1, 1/eps], hence the factor eps),

and the constant d makes the relative error sqrt(x) R(x) - 1 equioscillate
between -delta and +delta.  The partial fractions

    R(x) = a_0 + sum_l a_l / (x + sigma_l),

with sigma_l = eps c_{2l-1} are what the multishift solver consumes; for an
operator with spectrum in [lo, hi] the approximation is applied to N / hi
(see ``for_spectrum``).

Host-side set-up (numpy / scipy); the solves run on the GPU.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Rational:
    """a0 + sum_k a[k] / (x + shifts[k]) approximating x^(-1/2)."""
    a0: float
    a: np.ndarray
    shifts: np.ndarray
    delta: float  # max relative error on the interval it was built for
    lo: float
    hi: float

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self.a0 + np.sum(self.a[:, None] / (x.reshape(1, -1) + self.shifts[:, None]), axis=0).reshape(x.shape)


def _c_coefficients(n: int, eps: float) -> np.ndarray:
    from scipy.special import ellipj, ellipkm1

    m = 1.0 - eps                      # parameter k'^2
    Kp = ellipkm1(eps)                 # K(k') with 1 - k'^2 = eps, accurate for small eps
    u = np.arange(1, 2 * n + 1) * Kp / (2 * n + 1)
    sn, _, _, _ = ellipj(u, m)
    s2 = sn * sn
    return s2 / (1.0 - s2)             # c_1 .. c_2n


def _relative_error_extrema(f, lo: float, hi: float, npts: int = 20001):
    """min and max of f on [lo, hi]: a dense logarithmic grid, then each
    interior local extremum refined by a bounded scalar search."""
    from scipy.optimize import minimize_scalar

    t = np.linspace(np.log(lo), np.log(hi), npts)
    y = f(np.exp(t))
    vals = [y[0], y[-1]]
    for i in range(1, npts - 1):
        if (y[i] - y[i - 1]) * (y[i + 1] - y[i]) <= 0:
            sgn = 1.0 if y[i] > y[i - 1] else -1.0
            r = minimize_scalar(lambda s: -sgn * f(np.exp(np.array([s])))[0], bounds=(t[i - 1], t[i + 1]),
                                method="bounded", options={"xatol": 1e-12})
            vals.append(-sgn * r.fun)
    return min(vals), max(vals)


def inverse_sqrt(n: int, eps: float) -> Rational:
    """Zolotarev's degree-(n, n) best relative approximation of x^(-1/2) on [eps, 1]."""
    if not (0 < eps < 1) or n < 1:
        raise ValueError("need n >= 1 and 0 < eps < 1")
    c = eps * _c_coefficients(n, eps)  # back from [1, 1/eps] to [eps, 1]
    num, den = c[1::2], c[0::2]        # eps c_{2l}, eps c_{2l-1}

    def prod_form(x):
        x = np.asarray(x, dtype=np.float64)
        return np.prod((x[None, :] + num[:, None]) / (x[None, :] + den[:, None]), axis=0)

    lo_v, hi_v = _relative_error_extrema(lambda x: np.sqrt(x) * prod_form(x), eps, 1.0)
    d = 2.0 / (lo_v + hi_v)
    delta = (hi_v - lo_v) / (hi_v + lo_v)
    # partial fractions: residue of prod (x + num) / (x + den) at x = -den_l
    a = np.empty(n)
    for l in range(n):
        others = np.delete(den, l)
        a[l] = d * np.prod(num - den[l]) / np.prod(others - den[l])
    return Rational(a0=d, a=a, shifts=den.copy(), delta=float(delta), lo=eps, hi=1.0)


def for_spectrum(n: int, lo: float, hi: float) -> Rational:
    """N^(-1/2) ~ hi^(-1/2) R(N / hi) for a spectrum in [lo, hi]:
    a0 / sqrt(hi) + sum_l a_l sqrt(hi) / (N + hi sigma_l)."""
    r = inverse_sqrt(n, lo / hi)
    s = np.sqrt(hi)
    return Rational(a0=r.a0 / s, a=r.a * s, shifts=r.shifts * hi, delta=r.delta, lo=lo, hi=hi)

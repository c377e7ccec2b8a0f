"""Zolotarev coefficients of the rational approximation of x^(-1/2).

The pins do not reuse the construction: a rational function of type (n, n)
is the best uniform approximation (here of the relative error) exactly when
its error equioscillates at 2n + 2 points (Chebyshev's alternation theorem),
so a mistake in the elliptic-function coefficients, their scaling or the
normalisation shows up as a broken alternation pattern."""
import numpy as np
import pytest

from paper_2212_06635_amd import zolotarev as z


def _extrema(r, lo, hi, npts=400001):
    x = np.exp(np.linspace(np.log(lo), np.log(hi), npts))
    e = np.sqrt(x) * r(x) - 1.0
    idx = [0] + [i for i in range(1, npts - 1) if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) <= 0] + [npts - 1]
    return e[idx]


@pytest.mark.parametrize("n,eps", [(3, 1e-2), (6, 1e-4), (12, 1e-5)])
def test_relative_error_equioscillates(n, eps):
    r = z.inverse_sqrt(n, eps)
    ext = _extrema(r, eps, 1.0)
    assert len(ext) == 2 * n + 2
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))
    assert np.allclose(np.abs(ext), r.delta, rtol=1e-4)


def test_stieltjes_form_and_convergence():
    """Positive poles and residues (R(N) is then positive definite for N >= 0)
    and an error that falls geometrically with the number of poles."""
    deltas = []
    for n in (4, 8, 12, 16):
        r = z.inverse_sqrt(n, 1e-5)
        assert r.a0 > 0 and np.all(r.a > 0) and np.all(r.shifts > 0)
        deltas.append(r.delta)
    ratios = np.array(deltas[1:]) / np.array(deltas[:-1])
    assert np.all(ratios < 1e-1) and np.all(ratios > 1e-4)


def test_spectrum_scaling():
    """for_spectrum approximates N^(-1/2) on [lo, hi] with the same relative error."""
    lo, hi = 3e-4, 2.5
    r = z.for_spectrum(12, lo, hi)
    lam = np.exp(np.linspace(np.log(lo), np.log(hi), 100001))
    err = np.abs(np.sqrt(lam) * r(lam) - 1.0)
    assert err.max() <= r.delta * (1 + 1e-6)
    assert r.shifts.min() < lo < hi < r.shifts.max() * 10


def test_arguments_validated():
    for n, eps in ((0, 1e-3), (4, 0.0), (4, 1.0), (4, -1e-3)):
        with pytest.raises(ValueError):
            z.inverse_sqrt(n, eps)


"""Pins of the oracle's special functions against library routines and closed forms."""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import oracle


@pytest.mark.parametrize("nu", [1 / 3, 2 / 3, 5 / 3])
@pytest.mark.parametrize("x", [1e-12, 1e-6, 1e-3, 0.1, 1.0, 5.0, 30.0, 200.0])
def test_bessel_k_vs_scipy(nu, x):
    assert oracle.bessel_k(nu, x) == pytest.approx(sp.kv(nu, x), rel=2e-14)


@pytest.mark.parametrize("x", [1e-9, 1e-3, 0.5, 3.0, 40.0])
def test_int_bessel_k13_vs_quadrature(x):
    ref = si.quad(lambda z: sp.kve(1 / 3, z) * np.exp(-(z - x)), x, np.inf, epsabs=0, epsrel=1e-13,
                  limit=400)[0] * np.exp(-x)
    assert oracle.int_bessel_k(1 / 3, x) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("x", [1e-4, 0.2, 2.0, 9.0])
def test_int_k53_identity(x):
    """int_x^inf K_{5/3} = 2 K_{2/3}(x) - IntK_{1/3}(x) (recurrence K_{nu-1} + K_{nu+1} = -2 K_nu')."""
    lhs = oracle.int_bessel_k(5 / 3, x)
    rhs = 2 * sp.kv(2 / 3, x) - oracle.int_bessel_k(1 / 3, x)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("mu,nu", [(1, 2 / 3), (2, 1 / 3), (3, 2 / 3), (3, 1 / 3), (2, 2 / 3)])
def test_mellin_moments(mu, nu):
    """int_0^inf z^(mu-1) K_nu(z) dz = 2^(mu-2) Gamma((mu-nu)/2) Gamma((mu+nu)/2), integrated
    with the oracle's K_nu on a log grid (t = ln z, trapezoid)."""
    t = np.linspace(math.log(1e-45), math.log(80.0), 9001)
    z = np.exp(t)
    f = np.array([oracle.bessel_k(nu, v) for v in z]) * z ** mu
    val = np.trapezoid(f, t)
    exact = 2 ** (mu - 2) * math.gamma((mu - nu) / 2) * math.gamma((mu + nu) / 2)
    assert val == pytest.approx(exact, rel=1e-8)


@pytest.mark.parametrize("x", [0.0, 0.3, 1.0, 2.5, 6.0, 15.0])
def test_scorer_gi_prime_vs_mpmath(x):
    mp.mp.dps = 30
    ref = float(mp.diff(mp.scorergi, x))
    assert oracle.scorer_gi_prime(x) == pytest.approx(ref, rel=1e-12, abs=1e-16)


@pytest.mark.parametrize("x", [1.5, 3.0, 4.5])
def test_scorer_gi_prime_vs_airy(x):
    """Gi(x) = Bi(x)/3 + Ai(x) int_0^x Bi - Bi(x) int_0^x Ai  =>  Gi'(x) = Bi'(x)/3 +
    Ai'(x) int_0^x Bi - Bi'(x) int_0^x Ai (variation of parameters for y'' - x y = -1/pi)."""
    mp.mp.dps = 30
    ai, aip, bi, bip = sp.airy(x)
    iai = float(mp.quad(mp.airyai, [0, x]))      # scipy's itairy is only ~1e-8 accurate
    ibi = float(mp.quad(mp.airybi, [0, x]))
    ref = bip / 3 + aip * ibi - bip * iai
    assert oracle.scorer_gi_prime(x) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("x", [60.0, 300.0, 1e4])
def test_scorer_gi_prime_asymptote(x):
    """Gi'(x) ~ -(1/(pi x^2)) (1 + 8/x^3 + 280/x^6) for large x."""
    ref = -1 / (math.pi * x * x) * (1 + 8 / x ** 3 + 280 / x ** 6)
    assert oracle.scorer_gi_prime(x) == pytest.approx(ref, rel=1e-11)

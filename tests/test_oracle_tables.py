"""Error of the table specification against direct quadrature (the oracle's own build of
the tables, which the GPU build must reproduce to rounding)."""
import numpy as np
import pytest

import oracle


def test_bessel_table(otab):
    rng = np.random.default_rng(1)
    for x in np.exp(rng.uniform(np.log(1e-14), np.log(600), 300)):   # K(x) underflows past ~700
        ref = np.array([oracle.bessel_k(1 / 3, x), oracle.bessel_k(2 / 3, x), oracle.int_bessel_k(1 / 3, x)])
        assert np.max(np.abs(otab.bessel(x) / ref - 1)) < 1e-9


def test_ncs_rate_table(otab):
    rng = np.random.default_rng(2)
    for chi in np.exp(rng.uniform(np.log(1e-7), np.log(1e3), 60)):
        Ia, Ib = otab.ncs_rate(chi)
        # below chi = 1e-6 the spec extrapolates Ia linearly: relative error ~ chi
        assert Ia == pytest.approx(oracle.ncs_Ia(chi), rel=2e-8 if chi >= 1e-6 else 1e-6)
        assert Ib == pytest.approx(oracle.ncs_Ib(chi), rel=2e-6 if chi < 1e-6 else 2e-7)
    assert otab.ncs_rate(0.0) == (0.0, 0.0)


def test_nbw_rate_table(otab):
    rng = np.random.default_rng(3)
    for chi in np.exp(rng.uniform(np.log(0.05), np.log(1e3), 40)):
        Ja, Jb = otab.nbw_rate(chi)
        assert Ja == pytest.approx(oracle.nbw_Ja(chi), rel=1e-8)
        assert Jb == pytest.approx(oracle.nbw_Jb(chi), rel=1e-8)
    assert otab.nbw_rate(0.04) == (0.0, 0.0)


def test_vb_table(otab):
    rng = np.random.default_rng(4)
    for chi in np.exp(rng.uniform(np.log(1e-4), np.log(1e3), 40)):
        assert np.max(np.abs(otab.vb_M(chi) - oracle.vb_M(chi))) < 1e-7
    assert np.array_equal(otab.vb_M(1e-5), [4.0, 7.0])


@pytest.mark.parametrize("chi", [1e-5, 3e-3, 0.1, 0.8, 4.0, 10.0, 100.0])
def test_ncs_inverse_cdf(otab, chi):
    """CDF(y | s) = [A(y) - s B(y)] / [Ia - s Ib] at the sampled y equals the target r."""
    Ia, Ib = oracle.ncs_Ia(chi), oracle.ncs_Ib(chi)
    tol = 1.5e-5 if chi <= 10 else 1e-4
    for s in (-1.0, 0.4, 1.0):
        for r in (1e-5, 0.03, 0.3, 0.5, 0.77, 0.99, 0.99999):
            t = otab.ncs_sample_t(chi, s, r)
            u = 1.5 * chi * t ** 3
            y = u / (1 + u)
            c = (oracle.ncs_A(chi, y) - s * oracle.ncs_B(chi, y)) / (Ia - s * Ib)
            assert abs(c - r) < tol, (s, r, c)


@pytest.mark.parametrize("chi", [0.05, 0.4, 2.0, 10.0, 100.0])
def test_nbw_inverse_cdf(otab, chi):
    Ja, Jb = oracle.nbw_Ja(chi), oracle.nbw_Jb(chi)
    tol = 2e-5 if chi <= 10 else 1e-4
    for xi3 in (-1.0, 0.0, 0.8):
        for r in (0.01, 0.2, 0.5, 0.64, 0.95):
            d = otab.nbw_sample_delta(chi, xi3, r)
            c = (oracle.nbw_Ka(chi, d) - xi3 * oracle.nbw_Kb(chi, d)) / (Ja - xi3 * Jb)
            assert abs(c - r) < tol, (xi3, r, c)
        # symmetric spectrum: r and 1 - r map to delta and 1 - delta
        assert otab.nbw_sample_delta(chi, xi3, 0.3) == pytest.approx(1 - otab.nbw_sample_delta(chi, xi3, 0.7),
                                                                      abs=1e-12)


def test_sampler_monotone(otab):
    for chi in (1e-3, 0.5, 7.0):
        ts = [otab.ncs_sample_t(chi, 0.5, r) for r in np.linspace(1e-6, 1 - 1e-6, 400)]
        assert np.all(np.diff(ts) > 0)

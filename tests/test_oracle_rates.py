"""Pins of the oracle's NCS / NBW / VB rate integrals and spin/polarisation functions.

Every value here comes from something other than the oracle's own formula: closed-form
limits, textbook expansions, the paper's printed constants and fits (tests/golden), an
alternative form of the same integral evaluated with scipy, or a sum rule that links two
different equations of the paper.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SQ3 = math.sqrt(3.0)


def ik13(x):
    return oracle.int_bessel_k(1 / 3, x)


# ----------------------------------------------------------------------------- NCS rates
@pytest.mark.parametrize("chi", [0.01, 0.3, 2.0, 20.0])
def test_ncs_Ia_by_parts_with_scipy(chi):
    """Ia = int (1+u)^-3 [-(1+u) IntK13(u') + (2+2u+u^2) K23(u')] du.  Integrating the
    IntK13 term by parts removes it: int IntK13(u')/(1+u)^2 du = pi/sqrt3 -
    (2/(3chi)) int K13(u')/(1+u) du, so Ia follows from scipy's K_nu alone."""
    c = 2 / (3 * chi)
    f1 = lambda u: sp.kv(1 / 3, c * u) / (1 + u)
    f2 = lambda u: (2 + 2 * u + u * u) * sp.kv(2 / 3, c * u) / (1 + u) ** 3
    pts = [0, 1e-6, 1e-3, 0.1 * chi, chi, 10 * chi, 60 * chi]
    q1 = sum(si.quad(f1, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    q2 = sum(si.quad(f2, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    ref = c * q1 - math.pi / SQ3 + q2
    assert oracle.ncs_Ia(chi) == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("chi", [1e-3, 0.3, 2.0, 20.0])
def test_ncs_Ib_vs_scipy(chi):
    c = 2 / (3 * chi)
    f = lambda u: u * sp.kv(1 / 3, c * u) / (1 + u) ** 3
    pts = [0, 1e-3 * chi, 0.1 * chi, chi, 10 * chi, 60 * chi]
    ref = sum(si.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    assert oracle.ncs_Ib(chi) == pytest.approx(ref, rel=1e-10)


def test_ncs_classical_photon_number():
    """chi -> 0: total rate -> 5 alpha chi / (2 sqrt3 xi_L gamma), i.e. Ia -> 5 pi chi / 2,
    and Ib -> (9 chi^2/4) int z K13 = 3 pi chi^2 / 4 (Mellin moments)."""
    prev = 1.0
    for chi in (1e-3, 1e-4, 1e-5):
        d = abs(oracle.ncs_Ia(chi) / (2.5 * math.pi * chi) - 1)
        assert d < 1.5 * chi and d < prev
        prev = d
        assert oracle.ncs_Ib(chi) / (0.75 * math.pi * chi * chi) == pytest.approx(1, abs=10 * chi)


@pytest.mark.parametrize("chi", [1e-4, 3e-4])
def test_larmor_power_and_first_quantum_correction(chi):
    """Emitted power / (2/3) alpha chi^2 / xi_L (the classical limit of Sec. III.A.1)
    = 1 - (55 sqrt3/16) chi + 48 chi^2 + O(chi^3)."""
    g = oracle.ncs_power_ratio(chi)
    assert g == pytest.approx(1 - 55 * SQ3 / 16 * chi + 48 * chi * chi, abs=600 * chi ** 3)


def test_paper_q_fits():
    """The two approximations of q(chi) printed in Sec. III.A.2 track the exact power
    ratio (loose pin: fit A within 1.5 %, fit B within 13 % for chi in [1e-3, 50])."""
    A, B = GOLD["q_fit_A"], GOLD["q_fit_B"]
    for chi in np.geomspace(1e-3, 50, 25):
        g = oracle.ncs_power_ratio(chi)
        fa = (1 + A["coef"][0] * (1 + chi) * math.log(1 + A["coef"][1] * chi) + A["coef"][2] * chi ** 2) ** A["power"]
        fb = (1 + B["coef"][0] * chi + B["coef"][1] * chi ** 2) ** B["power"]
        assert abs(fa / g - 1) < 0.015, (chi, g, fa)
        assert abs(fb / g - 1) < 0.13, (chi, g, fb)


def test_sokolov_ternov_limits():
    """Radiative T-BMT integrals: psi3/psi1 -> 8/(5 sqrt3) and psi1 -> (15 pi/8) chi^3
    as chi -> 0 (Mellin moments of K23, K13 with z^2).  The paper quotes ~92.5 %."""
    st = 8 / (5 * SQ3)
    psi = oracle.rbmt_psi(1e-5)
    assert psi[2] / psi[0] == pytest.approx(st, abs=2e-5)
    assert psi[0] / (15 * math.pi / 8 * 1e-15) == pytest.approx(1, abs=20 * 1e-5)   # O(chi) correction ~ -11 chi
    assert abs(st - GOLD["sokolov_ternov_degree_approx"]["value"]) < 0.002
    # finite chi lowers the equilibrium degree monotonically
    vals = [oracle.rbmt_psi(c)[2] / oracle.rbmt_psi(c)[0] for c in (1e-3, 0.1, 1.0, 10.0)]
    assert all(a > b for a, b in zip(vals[:-1], vals[1:]))


@pytest.mark.parametrize("chi", [0.05, 1.0])
def test_psi1_psi3_vs_scipy(chi):
    c = 2 / (3 * chi)
    pts = [0, 0.1 * chi, chi, 10 * chi, 60 * chi]
    for k, nu in ((0, 2 / 3), (2, 1 / 3)):
        f = lambda u: u * u / (1 + u) ** 3 * sp.kv(nu, c * u)
        ref = sum(si.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
        assert oracle.rbmt_psi(chi)[k] == pytest.approx(ref, rel=1e-10)


# ------------------------------------------------------------ NCS spin / polarisation forms
def _triad(rng):
    n = rng.normal(size=3); n /= np.linalg.norm(n)
    a = rng.normal(size=3); a -= n * (a @ n); a /= np.linalg.norm(a)
    return a, np.cross(n, a), n


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_F0_equals_sqa_form_and_sums_to_wspin2():
    """F0 of eq. (F0) equals 4 (w + f.S_i + g.S_f) with w, f, g written from the SQA form
    of the paper (Bessel functions in the order of eqs. (F0)/(Wspin2), f = -u K13 b);
    summing over S_f = +-zeta gives 8 (w + f.S_i), the bracket of eq. (Wspin2)."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        chi = 10 ** rng.uniform(-2, 1.3)
        u = 10 ** rng.uniform(-3, 1.5)
        a, b, n = _triad(rng)
        Si, Sf = _unit(rng), _unit(rng)
        up = 2 * u / (3 * chi)
        I, K1, K2 = ik13(up), sp.kv(1 / 3, up), sp.kv(2 / 3, up)
        w = -(1 + u) * I + (2 + 2 * u + u * u) * K2
        f = -u * K1 * b
        g = -(1 + u) * (I - 2 * K2) * Si - u * (1 + u) * K1 * b - u * u * (I - K2) * (Si @ n) * n
        F = oracle.ncs_F(u, chi, Si, Sf, a, b, n)
        assert F[0] == pytest.approx(4 * (w + f @ Si + g @ Sf), rel=1e-11, abs=1e-12 * abs(w))
        z = _unit(rng)
        tot = oracle.ncs_F(u, chi, Si, z, a, b, n)[0] + oracle.ncs_F(u, chi, Si, -z, a, b, n)[0]
        wspin2 = -(1 + u) * I + (2 + 2 * u + u * u) * K2 - u * (Si @ b) * K1
        assert tot == pytest.approx(8 * wspin2, rel=1e-11)


def test_F_defines_a_positive_density_matrix():
    """(W_R/2)(F0 + xi.F) is a probability for every photon state |xi| <= 1, so
    F0 >= |(F1,F2,F3)| for all electron spins; F0 >= 0."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        chi = 10 ** rng.uniform(-3, 1.5)
        u = 10 ** rng.uniform(-4, 2)
        a, b, n = _triad(rng)
        F = oracle.ncs_F(u, chi, _unit(rng), _unit(rng), a, b, n)
        assert F[0] >= -1e-12 * abs(F).max()
        assert np.linalg.norm(F[1:]) <= F[0] * (1 + 1e-9) + 1e-14 * abs(F).max()


def _mean_stokes_unpolarised(chi, weight_energy):
    """Spin-averaged, S_f-summed <xi3> = int F3 / int F0 over the spectrum, using the
    oracle's F at S_i = +-S, S_f = +-zeta (for any S, zeta)."""
    rng = np.random.default_rng(3)
    a, b, n = _triad(rng)
    S, z = _unit(rng), _unit(rng)
    t = np.linspace(1e-4, 60 ** (1 / 3), 1500)
    num = den = 0.0
    vals = []
    for tt in t:
        u = 1.5 * chi * tt ** 3
        acc = np.zeros(4)
        for si_ in (S, -S):
            for sf in (z, -z):
                acc += oracle.ncs_F(u, chi, si_, sf, a, b, n)
        jac = 4.5 * chi * tt * tt / (1 + u) ** 3 * (u / (1 + u) if weight_energy else 1.0)
        vals.append(acc * jac)
    vals = np.array(vals)
    return np.trapezoid(vals[:, 3], t) / np.trapezoid(vals[:, 0], t), \
        np.trapezoid(vals[:, 1], t) / np.trapezoid(vals[:, 0], t), \
        np.trapezoid(vals[:, 2], t) / np.trapezoid(vals[:, 0], t)


def test_classical_linear_polarisation_of_ncs_photons():
    """chi -> 0, unpolarised electrons: <xi3> = int K23 / int (2K23 - IntK13) = 3/5
    counted per photon and 3/4 weighted by energy (Mellin moments); xi1 = xi2 = 0.
    The paper quotes a linear polarisation degree of about 60 %."""
    x3, x1, x2 = _mean_stokes_unpolarised(1e-4, False)
    assert x3 == pytest.approx(0.6, abs=2e-3)
    assert abs(x1) < 1e-10 and abs(x2) < 1e-10
    assert abs(x3 - GOLD["lp_gamma_xi3_approx"]["value"]) < 0.01
    e3, _, _ = _mean_stokes_unpolarised(1e-4, True)
    assert e3 == pytest.approx(0.75, abs=2e-3)


def test_longitudinal_spin_gives_circular_photons():
    """For S_i = n (longitudinal), the S_f-summed F2 = 4u(S_i.n)[(2+u)K23 - IntK13] != 0
    (circularly polarised photons from longitudinally polarised electrons, Sec. V.B)."""
    rng = np.random.default_rng(5)
    a, b, n = _triad(rng)
    z = _unit(rng)
    chi, u = 0.5, 0.3
    F = oracle.ncs_F(u, chi, n, z, a, b, n) + oracle.ncs_F(u, chi, n, -z, a, b, n)
    up = 2 * u / (3 * chi)
    ref = 2 * 4 * u * ((2 + u) * sp.kv(2 / 3, up) - ik13(up))
    assert F[2] == pytest.approx(ref, rel=1e-11)
    assert F[2] > 0


# ----------------------------------------------------------------------------- NBW
@pytest.mark.parametrize("chi", [0.3, 1.0, 8.0, 100.0, 900.0])
def test_nbw_J_vs_scipy(chi):
    def rho(d):
        return 2 / (3 * chi * d * (1 - d))
    fa = lambda d: ik13(rho(d)) + (d * d + (1 - d) ** 2) / (d * (1 - d)) * sp.kv(2 / 3, rho(d))
    fb = lambda d: sp.kv(2 / 3, rho(d))
    # at large chi the spectrum switches on at delta ~ 1/chi: give quad those breakpoints
    pts = sorted({1e-12, 0.5} | {v for v in (0.1 / chi, 1 / chi, 10 / chi) if v < 0.5})
    ja = 2 * sum(si.quad(fa, a, b, epsabs=0, epsrel=1e-11, limit=300)[0] for a, b in zip(pts[:-1], pts[1:]))
    jb = 2 * sum(si.quad(fb, a, b, epsabs=0, epsrel=1e-12, limit=300)[0] for a, b in zip(pts[:-1], pts[1:]))
    assert oracle.nbw_Ja(chi) == pytest.approx(ja, rel=1e-9)
    assert oracle.nbw_Jb(chi) == pytest.approx(jb, rel=1e-10)


def test_nbw_small_chi_asymptote_and_polarisation_ratio():
    """chi -> 0: W eps xi_L/alpha -> (3 sqrt3/(16 sqrt2)) chi exp(-8/(3chi)) and
    Jb/Ja -> 1/3 (IntK13 ~ K23 at large argument, r(1/2) = 2): photons polarised along
    E_red pair at half the rate of the orthogonal state."""
    prev = 1.0
    for chi in (0.1, 0.05, 0.02):
        T = oracle.nbw_Ja(chi) / (SQ3 * math.pi)
        asym = 3 * SQ3 / (16 * math.sqrt(2)) * chi * math.exp(-8 / (3 * chi))
        d = abs(T / asym - 1)
        assert d < 0.2 * chi and d < prev
        prev = d
        assert oracle.nbw_Jb(chi) / oracle.nbw_Ja(chi) == pytest.approx(1 / 3, abs=0.1 * chi)


def test_nbw_delta_symmetry():
    for chi in (0.2, 3.0):
        Ja = oracle.nbw_Ja(chi)
        for d in (0.1, 0.3, 0.45):
            assert oracle.nbw_Ka(chi, d) + oracle.nbw_Ka(chi, 1 - d) == pytest.approx(Ja, rel=1e-12)


def test_nbw_G_sum_rules_and_positivity():
    """Summing G0 + xi.G over S_- = +-zeta gives 2 (C + S_+.D) with C, D of eq. (BWposAxis);
    over S_+ gives 2 (C + S_-.D') with D' of eq. (BWeleAxis); every state has a
    non-negative weight."""
    rng = np.random.default_rng(21)
    for _ in range(60):
        chi = 10 ** rng.uniform(-0.5, 1.2)
        d = rng.uniform(0.02, 0.98)
        a, b, v = _triad(rng)
        xi = _unit(rng) * rng.uniform(0, 1)
        rho = 2 / (3 * chi * d * (1 - d))
        I, K1, K2 = ik13(rho), sp.kv(1 / 3, rho), sp.kv(2 / 3, rho)
        ep, em = d, 1 - d
        Cc = I + (em * em + ep * ep) / (em * ep) * K2 - xi[2] * K2
        D = (-(1 / ep - xi[2] / em) * K1 * b - xi[0] / em * K1 * a
             + xi[1] * ((ep * ep - em * em) / (em * ep) * K2 + I / ep) * v)
        Dp = ((1 / em - xi[2] / ep) * K1 * b + xi[0] / ep * K1 * a
              - xi[1] * ((ep * ep - em * em) / (em * ep) * K2 - I / em) * v)
        Sp, Sm, z = _unit(rng), _unit(rng), _unit(rng)
        wsum = lambda s1, s2: (lambda G: G[0] + xi @ G[1:])(oracle.nbw_G(d, chi, s1, s2, a, b, v))
        assert wsum(Sp, z) + wsum(Sp, -z) == pytest.approx(2 * (Cc + Sp @ D), rel=1e-10, abs=1e-13 * Cc)
        assert wsum(z, Sm) + wsum(-z, Sm) == pytest.approx(2 * (Cc + Sm @ Dp), rel=1e-10, abs=1e-13 * Cc)
        assert wsum(Sp, Sm) >= -1e-12 * Cc


# ----------------------------------------------------------------------------- VB
def test_vb_low_chi_constants():
    M = oracle.vb_M(1e-3)
    assert M[0] == pytest.approx(GOLD["vb_low_chi_M_plus"]["value"], abs=3e-6)
    assert M[1] == pytest.approx(GOLD["vb_low_chi_M_minus"]["value"], abs=3e-6)
    assert M[0] - M[1] == pytest.approx(GOLD["vb_low_chi_phase_factor"]["value"], abs=6e-6)


@pytest.mark.parametrize("chi", [0.5, 3.0, 20.0])
def test_vb_M_vs_scipy_quadrature(chi):
    def core(v):
        x = 4 / ((1 - v * v) * chi)
        X = x ** (2 / 3)
        return math.pi * X * X * oracle.scorer_gi_prime(X)
    mp_ = -11.25 * si.quad(lambda v: (1 - v * v) * 0.5 * (1 + v * v / 3) * core(v), 0, 1, epsabs=1e-14, limit=200)[0]
    mm_ = -11.25 * si.quad(lambda v: (1 - v * v) * (1 - v * v / 3) * core(v), 0, 1, epsabs=1e-14, limit=200)[0]
    M = oracle.vb_M(chi)
    assert M[0] == pytest.approx(mp_, rel=1e-9, abs=1e-12)
    assert M[1] == pytest.approx(mm_, rel=1e-9, abs=1e-12)

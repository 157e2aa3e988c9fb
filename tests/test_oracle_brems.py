"""Pins of the bremsstrahlung oracle (Sec. III.E) to results it does not compute itself:
the Coulomb correction against the series it fits, the screening functions against the
unscreened Bethe-Heitler limit, the cross-section in complete screening against Tsai's
closed form and the published radiation lengths of aluminium, copper and lead, the tables
against direct quadrature, and the Monte Carlo step against its defining probabilities."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import oracle.brems as BR

R0 = oracle.ALPHA * oracle.XI_L
ALPHA = oracle.ALPHA


def test_coulomb_correction_fits_its_series():
    """f(Z) = a^2 sum_n 1 / (n (n^2 + a^2)) (Davies, Bethe and Maximon); the fitted form is
    good to about 1e-4 for a <= 2/3."""
    n = np.arange(1, 2_000_001, dtype=np.float64)
    for Z in (5, 13, 29, 47, 74, 79, 92):
        a2 = (ALPHA * Z) ** 2
        series = a2 * (np.sum(1.0 / (n * (n * n + a2))) + 1.0 / (2.0 * n[-1] ** 2))
        assert abs(BR.coulomb_f(Z) - series) < 1.5e-4, (Z, BR.coulomb_f(Z), series)


def test_screening_functions_reach_the_unscreened_limit():
    """Without screening (gamma, eps >> 1), phi1 and psi1 become Bethe-Heitler's
    4 ln(2 E E' / (m k)) - 2, which in these variables reads 4 ln 200 - 2 - 4 ln gamma (resp.
    eps) apart from the ln Z terms the cross-section carries separately; phi1 - phi2 and
    psi1 - psi2 vanish."""
    target = 4.0 * math.log(200.0) - 2.0
    for g in (1e3, 1e4, 1e5):
        assert abs(BR.phi1(g) + 4.0 * math.log(g) - target) < 1e-3
        assert abs(BR.psi1(g) + 4.0 * math.log(g) - target) < 1e-3
        assert abs(BR.phi1(g) - BR.phi2(g)) < 1e-6 and abs(BR.psi1(g) - BR.psi2(g)) < 1e-6


def test_cross_section_without_screening_is_bethe_heitler():
    """At gamma, eps >> 1 the braces are Bethe-Heitler's unscreened ones with the Coulomb
    correction: (4/3 - 4/3 y + y^2) [4 (Z^2 + Z)(ln(2 E E'/(m k)) - 1/2) - 4 f Z^2] (at these
    points of any sign: the identity holds for the formula as printed)."""
    for Z, E, y in ((79, 10.0, 0.999), (13, 20.0, 0.9995), (29, 5.0, 0.9999)):
        g = 100.0 * y / ((1 - y) * E * Z ** (1 / 3))
        assert g > 500
        k, Ep = y * E, (1 - y) * E
        bh = (4 / 3 - 4 / 3 * y + y * y) * (4 * (Z * Z + Z) * (math.log(2 * E * Ep / k) - 0.5)
                                            - 4 * BR.coulomb_f(Z) * Z * Z)
        got = BR.bracket(y, E, Z)
        assert abs(got / bh - 1) < 2e-4, (Z, got, bh)


def _complete_screening_error(Z):
    """max relative deviation of the bracket at E -> inf from Tsai's complete-screening form
    (4/3 - 4/3 y + y^2) 4 [Z^2 (L_rad - f) + Z L'_rad] + 4/9 (1 - y)(Z^2 + Z),
    L_rad = ln(184.15 Z^-1/3), L'_rad = ln(1194 Z^-2/3)."""
    Lr, Lp, f = math.log(184.15 * Z ** (-1 / 3)), math.log(1194.0 * Z ** (-2 / 3)), BR.coulomb_f(Z)
    err = 0.0
    for y in (1e-4, 0.01, 0.3, 0.7, 0.95):
        want = (4 / 3 - 4 / 3 * y + y * y) * 4 * (Z * Z * (Lr - f) + Z * Lp) + 4 / 9 * (1 - y) * (Z * Z + Z)
        got = BR.y_dcs(y, 1e13, Z, R0) / (ALPHA * R0 * R0)
        err = max(err, abs(got / want - 1))
    return err


@pytest.mark.parametrize("Z", [5, 13, 29, 79, 92])
def test_complete_screening_limit(Z):
    assert _complete_screening_error(Z) < 2e-5


def test_planted_mistake_is_caught(monkeypatch):
    """A dropped factor 2/3 in phi2 (a plausible slip) fails the complete-screening pin."""
    monkeypatch.setattr(BR, "phi2", lambda g: BR.phi1(g) - 1.0 / (1.0 + 6.5 * g + 6.0 * g * g))
    assert _complete_screening_error(79) > 1e-3


@pytest.mark.parametrize("name,Z,A,X0", [("Al", 13, 26.9815, 24.01), ("Cu", 29, 63.546, 12.86),
                                         ("Pb", 82, 207.2, 6.37)])
def test_radiation_length(name, Z, A, X0):
    """Energy loss in complete screening, n int_0^1 y dsigma/dy dy = E n 4 alpha r0^2
    [Z^2 (L_rad - f) + Z L'_rad + (Z^2 + Z)/18]: the quadrature of the oracle's cross-section
    at E = 1e13 m c^2 reproduces the bracket, and without Tsai's (Z^2 + Z)/18 term (which his
    radiation length leaves out) gives the published radiation lengths (g/cm^2)."""
    E = 1e13
    val, _ = integrate.quad(lambda t: BR.y_dcs(math.exp(t), E, Z, R0) * math.exp(t), math.log(1e-12),
                            math.log(1 - 1e-9), limit=400, epsabs=0, epsrel=1e-11)
    val /= 4 * ALPHA * R0 * R0
    Lr, Lp, f = math.log(184.15 * Z ** (-1 / 3)), math.log(1194.0 * Z ** (-2 / 3)), BR.coulomb_f(Z)
    bracket = Z * Z * (Lr - f) + Z * Lp
    assert abs(val - (bracket + (Z * Z + Z) / 18.0)) < 1e-4 * bracket
    r0_cm = 2.8179403262e-13
    inv_x0 = 4 * ALPHA * r0_cm ** 2 * 6.02214076e23 / A * (val - (Z * Z + Z) / 18.0)
    assert abs(1.0 / inv_x0 / X0 - 1) < 2e-3, (name, 1.0 / inv_x0)


@pytest.fixture(scope="module")
def gold():
    # 1 MeV cut; density of gold in atoms per (c / omega_L)^3 at 1 um: 5.90e28 m^-3 (lambda/2pi)^3
    n = 5.90e28 * (1e-6 / (2 * math.pi)) ** 3
    mat = BR.Material(Z=79, n_atoms=n, x_lo=0.0, x_hi=1e9, k_cut=1.0 / 0.51099895)
    return mat, BR.build_tables(mat)


def test_tables_against_direct_quadrature(gold):
    mat, tab = gold
    assert np.all(np.diff(tab.cdf, axis=1) >= 0) and np.all(tab.sigma >= 0)
    for j in (1, 17, 80, 150, 255):
        E = math.exp(tab.lnE[j])
        lo, hi = math.log(mat.k_cut / E), math.log(1 - 1 / E)
        want, _ = integrate.quad(lambda t: BR.y_dcs(math.exp(t), E, mat.Z, R0), lo, hi, limit=400,
                                 epsabs=0, epsrel=1e-12)
        # the tables' fixed rule (8 points per u interval) against adaptive quadrature; the
        # kink where the cross-section reaches zero near the tip limits the fixed rule
        assert abs(tab.sigma[j] / want - 1) < 2e-8, j
        # the cumulative values at three interior nodes
        for i in (10, 64, 120):
            yu = BR.y_of(mat.k_cut, E, i / (BR.NU - 1))
            part, _ = integrate.quad(lambda t: BR.y_dcs(math.exp(t), E, mat.Z, R0), lo, math.log(yu),
                                     limit=400, epsabs=0, epsrel=1e-12)
            assert abs(tab.cdf[j, i] / part - 1) < 2e-8, (j, i)
    # between nodes sigma is the linear interpolant in ln E, close to the direct value
    E = math.exp(0.5 * (tab.lnE[100] + tab.lnE[101]))
    lo, hi = math.log(mat.k_cut / E), math.log(1 - 1 / E)
    want, _ = integrate.quad(lambda t: BR.y_dcs(math.exp(t), E, mat.Z, R0), lo, hi, limit=400)
    assert abs(BR.sigma_at(tab, E)[0] / want - 1) < 1e-3


def test_monte_carlo_step_statistics(gold):
    """1 GeV electrons in gold: the emitting fraction is 1 - exp(-n sigma ds); photon energies
    follow the cross-section above the cut (Kolmogorov-Smirnov against the direct CDF); each
    emission conserves energy and keeps the direction; electrons outside the slab are
    untouched; ids follow electron order."""
    mat0, tab = gold
    mat = BR.Material(mat0.Z, mat0.n_atoms, x_lo=-1.0, x_hi=1.0, k_cut=mat0.k_cut)
    n = 20000
    rng = np.random.default_rng(5)
    E0 = 1000.0 / 0.51099895
    pz = np.sqrt(E0 * E0 - 1.0)
    th = rng.normal(0, 1e-3, (n, 2))
    p = np.stack([pz * np.ones(n), pz * th[:, 0], pz * th[:, 1]], 1)
    p *= (pz / np.linalg.norm(p, axis=1))[:, None]
    st = {"x": np.where(np.arange(n) % 10 == 0, 5.0, 0.0), "y": np.zeros(n), "z": np.zeros(n),
          "px": p[:, 0], "py": p[:, 1], "pz": p[:, 2], "w": np.ones(n), "sx": np.zeros(n), "sy": np.zeros(n),
          "sz": np.zeros(n), "id": np.arange(n, dtype=np.uint64)}
    sig, _ = BR.sigma_at(tab, E0)
    dt = 0.2 / (mat.n_atoms * sig)                   # P = 1 - e^-0.2 (v ~ 1)
    sim = oracle.Sim(dt=dt, procs=0, seed=77, next_id=1 << 40, p_max=1.0)
    L = oracle.LeptonArrays.from_state(st)
    G = oracle.PhotonArrays.empty(n)
    status = BR.brems_step(sim, tab, mat, L, G, step=3)
    assert status == 0
    inside = st["x"] < 1.0
    P = -math.expm1(-mat.n_atoms * sig * (pz / E0) * dt)
    m = inside.sum()
    assert abs(G.count - m * P) < 4 * math.sqrt(m * P * (1 - P)), (G.count, m * P)
    v = L.view()
    out = ~inside
    for q in ("px", "py", "pz"):
        assert np.array_equal(v[q][out], st[q][out])
    g = G.view()
    k = np.sqrt(g["kx"] ** 2 + g["ky"] ** 2 + g["kz"] ** 2)
    assert np.all(k >= mat.k_cut * (1 - 1e-12))
    assert np.array_equal(g["id"], (1 << 40) + np.arange(G.count, dtype=np.uint64))
    emitted = np.flatnonzero(inside & (np.abs(v["px"] - st["px"]) > 0))
    assert len(emitted) == G.count
    Ea = np.sqrt(1 + v["px"][emitted] ** 2 + v["py"][emitted] ** 2 + v["pz"][emitted] ** 2)
    assert np.max(np.abs(Ea + k - E0) / E0) < 1e-12
    d_e = p[emitted] / pz
    d_g = np.stack([g["kx"], g["ky"], g["kz"]], 1) / k[:, None]
    assert np.max(np.abs(d_e - d_g)) < 1e-12
    # energy spectrum against the direct CDF of y at E0
    lo, hi = math.log(mat.k_cut / E0), math.log(1 - 1 / E0)
    tot, _ = integrate.quad(lambda t: BR.y_dcs(math.exp(t), E0, mat.Z, R0), lo, hi, limit=400)
    ys = np.sort(k / E0)
    cdf = np.array([integrate.quad(lambda t: BR.y_dcs(math.exp(t), E0, mat.Z, R0), lo, math.log(y), limit=200)[0]
                    for y in ys]) / tot
    ks = np.max(np.abs(cdf - (np.arange(1, len(ys) + 1) / len(ys))))
    assert ks < 1.63 / math.sqrt(len(ys)), ks        # 1 % level

"""Plain FP64 reference of the high-energy bremsstrahlung Monte Carlo (Sec. III.E) (TEST
INFRASTRUCTURE ONLY: used by tests/ to check the library's bremsstrahlung tables and step;
never by the product package).

Cross-section.  Per atom of charge Z, for an electron of total energy E (units of m c^2)
emitting a photon of energy k = y E, the differential cross-section of Sec. III.E (the
form of Tsai's review) is

    dsigma/dy = (alpha r0^2 / y) { (4/3 - 4/3 y + y^2) [Z^2 (phi1 - 4/3 ln Z - 4 f) + Z (psi1 - 8/3 ln Z)]
                                   + 2/3 (1 - y) [Z^2 (phi1 - phi2) + Z (psi1 - psi2)] }

with the screening functions of the Thomas-Fermi atom in Tsai's fitted form (his eqs.
3.38-3.41, which the paper names for Z >= 5), of gamma = 100 y / ((1 - y) E Z^(1/3)) and
eps = 100 y / ((1 - y) E Z^(2/3)):

    phi1(g) = 20.863 - 2 ln(1 + (0.55846 g)^2) - 4 (1 - 0.6 e^(-0.9 g) - 0.4 e^(-1.5 g))
    phi2(g) = phi1(g) - (2/3) / (1 + 6.5 g + 6 g^2)
    psi1(e) = 28.340 - 2 ln(1 + (3.621 e)^2) - 4 (1 - 0.7 e^(-8 e) - 0.3 e^(-29.2 e))
    psi2(e) = psi1(e) - (2/3) / (1 + 40 e + 400 e^2)

and the Coulomb correction f(Z) = a^2 [1/(1 + a^2) + 0.20206 - 0.0369 a^2 + 0.0083 a^4
- 0.002 a^6], a = alpha Z (the fit to a^2 sum_n 1 / (n (n^2 + a^2))).  Near the tip
(y -> 1 - 1/E) of heavy atoms the corrected bracket turns negative; the cross-section is
zero there.  r0 = alpha xi_L in the library's length unit c / omega_L.  Only Z >= 5 is covered: below, the paper switches
to tabulated scaled cross-sections that are not part of this build.

Tables (the algorithm's definition of sigma(E) and of the energy draw).  ln E on NE nodes
from ln E_lo = ln((k_cut + 1)(1 + 1e-6)) to ln E_HI.  The photon variable is the logit
t = ln(y / (1 - y)), in which the cross-section is smooth at both ends of its range (at
small y t ~ ln y; near y = 1 gamma = 100 e^t / (E Z^(1/3))); at energy E it runs from
t0 = logit(y_min), y_min = k_cut / E, to t1 = logit(y_max) = ln(E - 1), y_max = 1 - 1/E
(the electron keeps its rest energy), and u in [0, 1] maps to t0 + u (t1 - t0), on NU nodes
u_i = i / (NU - 1).  Row j holds the cumulative integrals C_j(u_i) = int_{y_min}^{y(u_i)}
dsigma/dy dy, each interval [u_(i-1), u_i] by one 8-point Gauss-Legendre rule in t
(integrand y (1 - y) dsigma/dy); sigma_j = C_j(1).  sigma(E) is linear in ln E between
nodes (0 below E_lo; above E_HI the last node and a status flag).  The energy draw r: the CDF of row pair (j, j+1) at the
weight w of E between them, F(u_i) = [(1-w) C_j(u_i) + w C_(j+1)(u_i)] / [(1-w) sigma_j +
w sigma_(j+1)], is inverted by locating r between consecutive nodes (the last i with
F(u_i) <= r) and interpolating u linearly; y = 1 / (1 + e^-t), t = t0 + u (t1 - t0) at the
electron's own E.

Monte Carlo step (the paper's direct sampling).  An electron inside the target slab
x_lo <= x < x_hi with sigma > 0 emits with probability P = 1 - exp(-n sigma ds),
ds = |v| dt (the paper prints the exponent without its minus sign; the reading is the
free-path probability).  Draws r = uniform4(id, step, STREAM_BREMS, seed): the event if
r[0] < P, the energy from r[1].  The photon (k = y E along the electron's velocity,
unpolarised, basis e1 = unit(y_hat - (y_hat.n) n), else of z_hat) is appended in electron
order with the next id; the electron keeps its direction with energy E (1 - y).  Photons
below k_cut are not produced (the paper's minimum-energy threshold).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle

STREAM_BREMS = 3
NE, NU = 256, 128
E_HI = 4.0e6                      # 2 TeV in m c^2
GL_X, GL_W = np.polynomial.legendre.leggauss(8)


def coulomb_f(Z: float, alpha: float = oracle.ALPHA) -> float:
    a2 = (alpha * Z) ** 2
    return a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2 - 0.002 * a2 * a2 * a2)


def phi1(g):
    return 20.863 - 2.0 * np.log(1.0 + (0.55846 * g) ** 2) - 4.0 * (1.0 - 0.6 * np.exp(-0.9 * g) - 0.4 * np.exp(-1.5 * g))


def phi2(g):
    return phi1(g) - (2.0 / 3.0) / (1.0 + 6.5 * g + 6.0 * g * g)


def psi1(e):
    return 28.340 - 2.0 * np.log(1.0 + (3.621 * e) ** 2) - 4.0 * (1.0 - 0.7 * np.exp(-8.0 * e) - 0.3 * np.exp(-29.2 * e))


def psi2(e):
    return psi1(e) - (2.0 / 3.0) / (1.0 + 40.0 * e + 400.0 * e * e)


def bracket(y, E, Z, alpha=oracle.ALPHA):
    """The braces of the cross-section (y dsigma/dy / (alpha r0^2)) as printed, any sign."""
    y = np.asarray(y, dtype=np.float64)
    g = 100.0 * y / ((1.0 - y) * E * Z ** (1.0 / 3.0))
    e = 100.0 * y / ((1.0 - y) * E * Z ** (2.0 / 3.0))
    lz, f = np.log(Z), coulomb_f(Z, alpha)
    p1, p2, s1, s2 = phi1(g), phi2(g), psi1(e), psi2(e)
    a = (4.0 / 3.0 - 4.0 / 3.0 * y + y * y) * (Z * Z * (p1 - 4.0 / 3.0 * lz - 4.0 * f) + Z * (s1 - 8.0 / 3.0 * lz))
    b = (2.0 / 3.0) * (1.0 - y) * (Z * Z * (p1 - p2) + Z * (s1 - s2))
    return a + b


def y_dcs(y, E, Z, r0, alpha=oracle.ALPHA):
    """y dsigma/dy per atom.  Near the tip (y -> 1 - 1/E) of heavy atoms the Coulomb
    correction drives the braces below zero, where no cross-section exists: zero there."""
    return alpha * r0 * r0 * np.maximum(bracket(y, E, Z, alpha), 0.0)


def dcs(y, E, Z, r0, alpha=oracle.ALPHA):
    """dsigma/dy per atom."""
    return y_dcs(y, E, Z, r0, alpha) / np.asarray(y, dtype=np.float64)


@dataclass
class Material:
    Z: int
    n_atoms: float          # atoms per (c / omega_L)^3
    x_lo: float
    x_hi: float
    k_cut: float            # lowest photon energy produced (m c^2)


@dataclass
class Tables:
    lnE: np.ndarray         # [NE]
    sigma: np.ndarray       # [NE]
    cdf: np.ndarray         # [NE][NU]  C_j(u_i) (not normalised)


def e_lo(k_cut: float) -> float:
    return (k_cut + 1.0) * (1.0 + 1e-6)


def t_range(k_cut: float, E: float):
    """logit(y_min), logit(y_max) at energy E."""
    ymin = k_cut / E
    return np.log(ymin / (1.0 - ymin)), np.log(E - 1.0)


def y_of(k_cut: float, E: float, u: float) -> float:
    t0, t1 = t_range(k_cut, E)
    return 1.0 / (1.0 + np.exp(-(t0 + u * (t1 - t0))))


def build_tables(mat: Material, xi_L: float = oracle.XI_L, alpha: float = oracle.ALPHA) -> Tables:
    r0 = alpha * xi_L
    lnE = np.log(e_lo(mat.k_cut)) + (np.log(E_HI) - np.log(e_lo(mat.k_cut))) * np.arange(NE) / (NE - 1)
    cdf = np.zeros((NE, NU))
    u = np.arange(NU) / (NU - 1)
    for j in range(NE):
        E = np.exp(lnE[j])
        t0, t1 = t_range(mat.k_cut, E)
        acc = 0.0
        for i in range(1, NU):
            a, b = t0 + (t1 - t0) * u[i - 1], t0 + (t1 - t0) * u[i]
            t = 0.5 * (a + b) + 0.5 * (b - a) * GL_X
            y = 1.0 / (1.0 + np.exp(-t))
            acc += 0.5 * (b - a) * float(np.sum(GL_W * y_dcs(y, E, mat.Z, r0, alpha) * (1.0 - y)))
            cdf[j, i] = acc
    return Tables(lnE, cdf[:, -1].copy(), cdf)


def locate(tab: Tables, E: float):
    """(j, w, clamped): node below E and the weight of node j+1; None below the table."""
    lnE = np.log(E)
    if lnE < tab.lnE[0]:
        return None
    pos = (lnE - tab.lnE[0]) / (tab.lnE[1] - tab.lnE[0])
    if pos >= NE - 1:
        return NE - 2, 1.0, pos > NE - 1
    j = int(np.floor(pos))
    return j, pos - j, False


def sigma_at(tab: Tables, E: float):
    """(sigma, clamped)."""
    loc = locate(tab, E)
    if loc is None:
        return 0.0, False
    j, w, cl = loc
    return (1.0 - w) * tab.sigma[j] + w * tab.sigma[j + 1], cl


def sample_u(tab: Tables, E: float, r: float) -> float:
    j, w, _ = locate(tab, E)
    F = ((1.0 - w) * tab.cdf[j] + w * tab.cdf[j + 1]) / ((1.0 - w) * tab.sigma[j] + w * tab.sigma[j + 1])
    i = 0
    while i < NU - 2 and F[i + 1] <= r:
        i += 1
    d = F[i + 1] - F[i]
    f = (r - F[i]) / d if d > 0 else 0.0
    f = min(max(f, 0.0), 1.0)
    return (i + f) / (NU - 1)


def photon_basis(n):
    for axis in (np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])):
        e = axis - np.dot(axis, n) * n
        nn = np.dot(e, e)
        if nn > 1e-12:
            return e / np.sqrt(nn)
    raise AssertionError("unreachable")


def brems_step(sim: "oracle.Sim", tab: Tables, mat: Material, L: "oracle.LeptonArrays",
               G: "oracle.PhotonArrays", step: int) -> int:
    """One bremsstrahlung step over the electrons of L (photons appended to G in electron
    order, ids from sim's counter).  Returns the status bits it raised (1: an electron above
    the table's top energy, 2: photon list full, 4: a probability above sim's p_max)."""
    status = 0
    dt, seed, n_at = sim.cfg.dt, sim.cfg.seed, mat.n_atoms
    for i in range(L.count):
        if not (mat.x_lo <= L.x[i] < mat.x_hi):
            continue
        p = np.array([L.px[i], L.py[i], L.pz[i]])
        pp = float(np.sqrt(np.dot(p, p)))
        E = float(np.sqrt(1.0 + pp * pp))
        sig, cl = sigma_at(tab, E)
        if cl:
            status |= 1
        if not sig > 0.0:
            continue
        P = -np.expm1(-n_at * sig * (pp / E) * dt)
        if P > sim.cfg.p_max:
            status |= 4
        r = oracle.uniform4(int(L.id[i]), step, STREAM_BREMS, seed)
        if not r[0] < P:
            continue
        y = y_of(mat.k_cut, E, sample_u(tab, E, r[1]))
        k = y * E
        nhat = p / pp
        Ep = E - k
        L.px[i], L.py[i], L.pz[i] = p * (np.sqrt(Ep * Ep - 1.0) / pp)
        pid = sim.cfg.next_id
        sim.cfg.next_id += 1
        if G.count >= len(G.x):
            status |= 2
            continue
        c = G.count
        G.x[c], G.y[c], G.z[c] = L.x[i], L.y[i], L.z[i]
        G.kx[c], G.ky[c], G.kz[c] = k * nhat
        G.w[c] = L.w[i]
        G.xi1[c] = G.xi2[c] = G.xi3[c] = 0.0
        G.e1x[c], G.e1y[c], G.e1z[c] = photon_basis(nhat)
        G.id[c] = pid
        G.alive[c] = 1
        G.count += 1
    return status

"""The spin- and polarisation-resolved emission functions F0..F3 of Sec. III.C.1 (eqs. F0-F3)
derived again from first principles and compared with the oracle's.

The photon emission amplitude of an electron in a constant crossed field (the field the
local-constant-field rates of Sec. III.C.1 are computed for) is evaluated with Volkov
states of the Dirac equation: a plane wave of wave vector k = (1, -1, 0, 0) and potential
eA = (0, 0, a1 phi, 0), phi = k.x.  The transverse and light-front momenta are conserved;
what remains is one integral over phi of a spinor matrix element that is quadratic in phi
against a phase that is cubic in phi, i.e. Airy functions.  Squaring the amplitude for
initial and final rest-frame spins S_i, S_f and summing over the photon's transverse
momentum gives the photon polarisation density matrix, whose Stokes parameters in the
basis (P1, P2) = (a - n(n.a), n x P1) follow from the density matrix printed in Sec.
III.C.2.  These must equal (F0, F1, F2, F3)(u, chi, S_i, S_f) up to one positive factor
that depends on u and chi only.  Nothing of the oracle enters the derivation: it is
Dirac matrices, spinors and Airy functions.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
       np.array([[1, 0], [0, -1]], complex)]
_I2, _Z2 = np.eye(2, dtype=complex), np.zeros((2, 2), complex)
G0 = np.block([[_I2, _Z2], [_Z2, -_I2]])
GV = [np.block([[_Z2, s], [-s, _Z2]]) for s in SIG]   # Dirac representation


def slash(v):
    """gamma^mu v_mu for a contravariant 4-vector v (metric +---)."""
    return G0 * v[0] - GV[0] * v[1] - GV[1] * v[2] - GV[2] * v[3]


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def spin2(S):
    """two-spinor c with c^+ sigma c = S (unit vector)"""
    th, ph = np.arccos(np.clip(S[2], -1, 1)), np.arctan2(S[1], S[0])
    return np.array([np.cos(th / 2), np.exp(1j * ph) * np.sin(th / 2)])


def u_spinor(p, S):
    """free positive-energy spinor (m = 1) of momentum p whose rest-frame spin is S: the
    pure boost of the rest spinor, Dirac representation, u-bar u = 2"""
    c = spin2(S)
    sp_ = sum(SIG[k] * p[k + 1] for k in range(3))
    return np.concatenate([np.sqrt(p[0] + 1) * c, sp_ @ c / np.sqrt(p[0] + 1)])


K = np.array([1.0, -1.0, 0.0, 0.0])   # laser wave vector (wave along -x), phi = t + x


def volkov(p, a1, x):
    """Volkov solution of (i dslash - e Aslash - 1) psi = 0 for eA = (0, 0, a1 phi, 0), spin
    +z, at the event x: [1 + kslash eAslash/(2 k.p)] u(p) exp(i S)"""
    phi = mdot(K, x)
    A = np.array([0.0, 0.0, a1 * phi, 0.0])
    kp = mdot(K, p)
    S = -mdot(p, x) - (mdot(p, A) * phi / 2 / kp) + (-(a1 * a1) * phi ** 3 / 3) / (2 * kp)
    # the phase above is -p.x - int_0^phi [p.eA/(k.p) - (eA)^2/(2 k.p)] dphi' for p_y = 0
    return (np.eye(4) + slash(K) @ slash(A) / (2 * kp)) @ u_spinor(p, np.array([0, 0, 1.0])) * np.exp(1j * S)


def test_volkov_state_solves_the_dirac_equation():
    """The plane-wave states the derivation uses are solutions of the Dirac equation in
    the field (checked by central differences), so their phase and spinor factor carry
    the charge convention of the amplitude."""
    a1, h = 0.3, 1e-5
    p = np.array([np.sqrt(1 + 0.4 ** 2 + 0.7 ** 2), 0.4, 0.0, 0.7])
    for x in (np.array([0.1, 0.2, -0.3, 0.5]), np.array([1.3, -0.4, 0.2, -0.1])):
        phi = mdot(K, x)
        A = np.array([0.0, 0.0, a1 * phi, 0.0])
        dpsi = []
        for mu in range(4):
            e = np.zeros(4)
            e[mu] = h
            dpsi.append((volkov(p, a1, x + e) - volkov(p, a1, x - e)) / (2 * h))
        psi = volkov(p, a1, x)
        # i gamma^mu d_mu with contravariant index on gamma: gamma^0 d_t + gamma^k d_k
        lhs = 1j * (G0 @ dpsi[0] + sum(GV[k] @ dpsi[k + 1] for k in range(3))) - slash(A) @ psi - psi
        assert np.abs(lhs).max() < 1e-7 * np.abs(psi).max()


def derived_F(u, chi, pairs, gamma=1e5, nq=1601):
    """(F0, F1, F2, F3) up to a common factor for each (S_i, S_f) in pairs, from the Volkov
    amplitude; also returns the frame (a, b, n) of the initial electron.  The local-field
    forms hold as gamma -> infinity; at gamma = 1e5 the difference is O(1/gamma) and the
    spinor arithmetic still keeps about ten digits."""
    p = np.array([gamma, np.sqrt(gamma * gamma - 1), 0.0, 0.0])
    kp = mdot(K, p)
    a1 = chi / kp                         # chi = |a1| (k.p) for this field
    s = u / (1 + u)                       # light-front photon fraction, u = s/(1 - s)
    kpl = s * (p[0] + p[1])
    ppl = (p[0] + p[1]) - kpl
    a_hat = -np.sign(a1) * np.array([0.0, 1.0, 0.0])   # d(kinetic momentum)/dphi ~ -eA'
    n_hat = np.array([1.0, 0.0, 0.0])
    b_hat = np.cross(n_hat, a_hat)
    a1s, ks = slash(np.array([0.0, 0.0, a1, 0.0])), slash(K)
    # photon transverse momentum q (along z; the y-component only shifts the emission
    # phase): q = qs sinh(t), trapezoid rule in t
    qs = 3 * max(s, 1e-3)
    t = np.linspace(-np.arcsinh(80.0), np.arcsinh(80.0), nq)
    q_all, w_all = qs * np.sinh(t), qs * np.cosh(t) * (t[1] - t[0])
    out = np.zeros((len(pairs), 4))
    ui = [u_spinor(p, Si) for Si, _ in pairs]
    for q, w in zip(q_all, w_all):
        kq = np.array([(kpl + q * q / kpl) / 2, (kpl - q * q / kpl) / 2, 0.0, q])
        pmn = (1 + q * q) / ppl
        pf = np.array([(ppl + pmn) / 2, (ppl - pmn) / 2, 0.0, -q])
        kpf = mdot(K, pf)
        V0 = pf[0] + kq[0] - p[0]                          # linear phase coefficient
        b3 = (a1 * a1 / 6) * (1 / kpf - 1 / kp)             # cubic phase coefficient
        z = V0 / (3 * b3) ** (1 / 3)
        if z > 150:
            continue
        ai, aip, _, _ = sp.airy(z)
        c = 2 * np.pi
        I0 = (3 * b3) ** (-1 / 3) * c * ai                  # int phi^j exp(i(V0 phi + b3 phi^3))
        I1 = (3 * b3) ** (-2 / 3) * (-1j) * c * aip
        I2 = -(3 * b3) ** (-1.0) * c * z * ai
        nq_ = kq[1:] / np.linalg.norm(kq[1:])
        e1 = a_hat - nq_ * (nq_ @ a_hat)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nq_, e1)
        ops = []
        for e in (e1, e2):
            es = slash(np.array([0.0, *e]))
            m1 = (a1s @ ks / (2 * kpf)) @ es + es @ (ks @ a1s / (2 * kp))
            m2 = a1s @ ks @ es @ ks @ a1s / (4 * kp * kpf)
            ops.append(es * I0 + m1 * I1 + m2 * I2)
        for j, (_, Sf) in enumerate(pairs):
            ub = u_spinor(pf, Sf).conj() @ G0
            M1, M2 = ub @ ops[0] @ ui[j], ub @ ops[1] @ ui[j]
            x = M1 * np.conj(M2)
            out[j] += w * np.array([abs(M1) ** 2 + abs(M2) ** 2, 2 * x.real, -2 * x.imag,
                                    abs(M1) ** 2 - abs(M2) ** 2])
    return out, a_hat, b_hat, n_hat


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("u,chi", [(0.05, 0.2), (0.3, 1.0), (2.0, 0.5), (8.0, 3.0), (30.0, 10.0)])
def test_F0_F3_equal_the_volkov_amplitude(u, chi):
    """Every term of eqs. (F0)-(F3), including F1 and the S_f-dependent parts of F2 and F3,
    against the squared Volkov amplitude for random unit spins: one common positive factor,
    then agreement to 5e-5 of the largest component (a dropped term, a wrong sign or a
    swapped S_i / S_f changes some component by O(1))."""
    rng = np.random.default_rng(int(100 * u + 7 * chi))
    pairs = [(_unit(rng), _unit(rng)) for _ in range(5)]
    pairs += [(np.array([0.0, 0.0, 1.0]), _unit(rng)), (_unit(rng), np.array([1.0, 0.0, 0.0]))]
    Fd, a, b, n = derived_F(u, chi, pairs)
    Fo = np.array([oracle.ncs_F(u, chi, Si, Sf, a, b, n) for Si, Sf in pairs])
    lam = (Fd * Fo).sum() / (Fo * Fo).sum()
    assert lam > 0
    assert np.abs(Fd - lam * Fo).max() < 5e-5 * np.abs(lam * Fo).max()


def test_volkov_pin_catches_a_planted_sign_slip():
    """The same comparison fails for the oracle's F with one S_f term of F1 flipped
    (the n.(S_f x S_i) term): the pin resolves single terms."""
    rng = np.random.default_rng(3)
    pairs = [(_unit(rng), _unit(rng)) for _ in range(5)]
    u, chi = 0.3, 1.0
    Fd, a, b, n = derived_F(u, chi, pairs)
    up = 2 * u / (3 * chi)
    K23 = sp.kv(2 / 3, up)
    Fo = []
    for Si, Sf in pairs:
        F = oracle.ncs_F(u, chi, Si, Sf, a, b, n)
        F[1] -= 2 * (2 * u * (2 + u) * (n @ np.cross(Sf, Si)) * K23)   # flip that term's sign
        Fo.append(F)
    Fo = np.array(Fo)
    lam = (Fd * Fo).sum() / (Fo * Fo).sum()
    assert np.abs(Fd - lam * Fo).max() > 1e-2 * np.abs(lam * Fo).max()

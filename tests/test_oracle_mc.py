"""Monte-Carlo pins of the oracle's NCS, NBW and VB steps.

The statistical tests use fixed seeds and 4.5-sigma acceptance bands.  What they pin:
  * the one-step mean spin change of emission + no-emission branches equals the
    radiative T-BMT drift -P[psi1 S + psi2 (S.beta) beta + psi3 n_B] (Sec. III.B.2) --
    this links the NCS Monte-Carlo (Sec. III.C.1) to a different equation of the paper;
  * the event fraction equals the total rate times dt;
  * the photon spectrum follows the rate integral (chi^2 against quadrature);
  * the mean photon Stokes vector equals int F / int F0;
  * energy-momentum bookkeeping of every event; ordering and ids of appended particles;
  * the VB rotation in a static crossed field against the paper's low-chi phase -3 D.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import ALPHA, XI_L

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SQ3 = math.sqrt(3.0)


def _beam_in_B(n, gamma, chi, S, seed_id0=0):
    """n electrons along +x with Lorentz factor gamma in a uniform B along z chosen so that
    chi_e = chi; returns leptons, E6 (fields per particle) and the frame (a, b, n)."""
    pm = math.sqrt(gamma * gamma - 1)
    B = chi / (XI_L * pm)
    st = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "px": np.full(n, pm), "py": np.zeros(n),
          "pz": np.zeros(n), "w": np.ones(n), "sx": np.full(n, S[0]), "sy": np.full(n, S[1]),
          "sz": np.full(n, S[2]), "id": np.arange(seed_id0, seed_id0 + n, dtype=np.uint64)}
    L = oracle.LeptonArrays.from_state(st, charge=-1)
    E6 = np.zeros(6 * n)
    E6[5::6] = B
    # electron: acceleration q beta x B = -(x x z) B = +y;  b = n x a = z
    return L, E6, (np.array([0, 1.0, 0]), np.array([0, 0, 1.0]), np.array([1.0, 0, 0]))


def _dt_for(P, gamma, chi, s=0.0):
    C = ALPHA / (SQ3 * math.pi * XI_L * gamma)
    return P / (C * (oracle.ncs_Ia(chi) - s * oracle.ncs_Ib(chi))), C


@pytest.mark.parametrize("chi", [0.3, 2.0])
def test_mean_spin_drift_equals_radiative_bmt(chi):
    gamma, n = 1000.0, 1_000_000
    psi = oracle.rbmt_psi(chi)
    for label, S in (("long", (1.0, 0, 0)), ("trans_a", (0, 1.0, 0)), ("trans_b", (0, 0, 1.0))):
        L, E6, (a, b, nn) = _beam_in_B(n, gamma, chi, S)
        s = np.array(S) @ b
        dt, C = _dt_for(0.03, gamma, chi, s)
        sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS, seed=77, next_id=1 << 40)
        sim.emit(L, E6, None, 3)
        dS = np.stack([L.sx[:n], L.sy[:n], L.sz[:n]]) - np.array(S)[:, None]
        mean, err = dS.mean(axis=1), dS.std(axis=1) / math.sqrt(n)
        Sv = np.array(S)
        drift = -C * (psi[0] * Sv + psi[1] * (Sv @ nn) * nn + psi[2] * b) * dt
        # the one-step no-emission normalisation adds O((C Ib dt)^2); allow it in the band
        extra = (C * oracle.ncs_Ib(chi) * dt) ** 2
        for k in range(3):
            assert abs(mean[k] - drift[k]) < 4.5 * err[k] + extra + 1e-12, (label, k, mean, drift, err)


def test_event_fraction_spectrum_and_kinematics():
    gamma, chi, n = 2000.0, 1.0, 400_000
    L, E6, (a, b, nn) = _beam_in_B(n, gamma, chi, (0, 0, -1.0))
    s = -1.0
    dt, C = _dt_for(0.04, gamma, chi, s)
    p0 = np.stack([L.px[:n], L.py[:n], L.pz[:n]]).copy()
    G = oracle.PhotonArrays.empty(n)
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS | oracle.PROC_NCS_STOKES, seed=5, next_id=1000)
    sim.emit(L, E6, G, 11)
    m = G.count
    assert abs(m - 0.04 * n) < 4.5 * math.sqrt(n * 0.04 * 0.96)
    # ids are consecutive in parent order, photons start at the parent position
    assert np.array_equal(G.id[:m], np.arange(1000, 1000 + m, dtype=np.uint64))
    assert sim.next_id == 1000 + m
    pf = np.stack([L.px[:n], L.py[:n], L.pz[:n]])
    emitted = np.where(np.abs(pf[0] - p0[0]) > 0)[0]
    assert len(emitted) == m
    k = np.stack([G.kx[:m], G.ky[:m], G.kz[:m]])
    # momentum is conserved to rounding at every event
    assert np.max(np.abs(pf[:, emitted] + k - p0[:, emitted])) < 1e-12 * np.abs(p0).max()
    # photon Stokes vectors are pure states; e1 is the unit acceleration direction
    xi = np.stack([G.xi1[:m], G.xi2[:m], G.xi3[:m]])
    assert np.allclose(np.linalg.norm(xi, axis=0), 1.0, atol=1e-12)
    assert np.allclose(G.e1y[:m], 1.0) and np.allclose(G.e1x[:m], 0.0)
    # final spins are unit vectors
    S = np.stack([L.sx[:n], L.sy[:n], L.sz[:n]])
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0, atol=1e-12)
    # spectrum: chi^2 of y in 12 quantile bins of the exact CDF [A - s B]/[Ia - s Ib]
    y = k[0] / p0[0, 0]
    Ia, Ib = oracle.ncs_Ia(chi), oracle.ncs_Ib(chi)
    edges = [0.0]
    for q in np.linspace(0, 1, 13)[1:-1]:
        lo, hi = 0.0, 1.0
        for _ in range(50):
            mid = 0.5 * (lo + hi)
            c = (oracle.ncs_A(chi, mid) - s * oracle.ncs_B(chi, mid)) / (Ia - s * Ib)
            lo, hi = (mid, hi) if c < q else (lo, mid)
        edges.append(0.5 * (lo + hi))
    edges.append(1.0)
    h, _ = np.histogram(y, bins=edges)
    chi2 = np.sum((h - m / 12) ** 2 / (m / 12))
    assert chi2 < 40, chi2      # 11 dof: P(chi2 > 40) ~ 4e-5


def test_mean_photon_stokes_matches_rate_integrals():
    """For unpolarised electrons (S = +-z equally) the mean Stokes vector of the emitted
    photons equals int F / int F0 over the spectrum, summed over final spins."""
    gamma, chi, n = 1000.0, 0.5, 600_000
    L, E6, (a, b, nn) = _beam_in_B(n, gamma, chi, (0, 0, 1.0))
    L.sz[: n // 2] = -1.0
    dt, C = _dt_for(0.04, gamma, chi, 0.0)
    G = oracle.PhotonArrays.empty(n)
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS | oracle.PROC_NCS_STOKES, seed=8, next_id=1)
    sim.emit(L, E6, G, 2)
    m = G.count
    xi = np.stack([G.xi1[:m], G.xi2[:m], G.xi3[:m]])
    mean, err = xi.mean(axis=1), xi.std(axis=1) / math.sqrt(m)
    # quadrature of the expectation in the variable t (u = 1.5 chi t^3)
    t = np.linspace(1e-4, 60 ** (1 / 3), 1200)
    acc = []
    for tt in t:
        u = 1.5 * chi * tt ** 3
        tot = np.zeros(4)
        for Si in ((0, 0, 1.0), (0, 0, -1.0)):
            Si = np.array(Si)
            z = np.array([0.3, -0.5, 0.81]); z /= np.linalg.norm(z)
            for Sf in (z, -z):
                tot += oracle.ncs_F(u, chi, Si, Sf, a, b, nn)
        acc.append(tot * 4.5 * chi * tt * tt / (1 + u) ** 3)
    acc = np.array(acc)
    expect = np.trapezoid(acc[:, 1:], t, axis=0) / np.trapezoid(acc[:, 0], t)
    assert np.all(np.abs(mean - expect) < 4.5 * err + 1e-4), (mean, expect, err)
    assert expect[2] > 0.5


def test_no_field_no_change():
    L, E6, _ = _beam_in_B(100, 500.0, 0.5, (0, 1.0, 0))
    E6[:] = 0
    before = L.view()
    sim = oracle.Sim(dt=0.1, procs=oracle.PROC_NCS, seed=1, next_id=1)
    sim.emit(L, E6, None, 0)
    after = L.view()
    for k in before:
        assert np.array_equal(before[k], after[k])


def _photons(n, eps, xi, e1=(0, 1.0, 0), k_dir=(1.0, 0, 0)):
    kd = np.array(k_dir) / np.linalg.norm(k_dir)
    st = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n),
          "kx": np.full(n, eps * kd[0]), "ky": np.full(n, eps * kd[1]), "kz": np.full(n, eps * kd[2]),
          "w": np.ones(n), "xi1": np.full(n, xi[0]), "xi2": np.full(n, xi[1]), "xi3": np.full(n, xi[2]),
          "e1x": np.full(n, e1[0]), "e1y": np.full(n, e1[1]), "e1z": np.full(n, e1[2]),
          "id": np.arange(n, dtype=np.uint64), "alive": np.ones(n, np.uint8)}
    return oracle.PhotonArrays.from_state(st)


def test_vb_crossed_field_rotation():
    """Static crossed field E_y = -B_z (the VB example of Sec. III.F): a photon along +x
    sees E_red = 2 E_y y_hat, its basis stays fixed and (xi1, xi2) rotate by the same
    delta phi every step: xi1 = cos(N dphi), xi2 = sin(N dphi), xi3 unchanged.  At small
    chi the phase per unit length is -3 D (the paper's low-field value)."""
    eps = 1000.0 / 0.51099895      # 1 GeV
    for Ey, label in ((100.0, "paper"), (0.2, "low")):
        spec = {"kind": oracle.FIELD_CONST, "e0": (0, Ey, 0), "b0": (0, 0, -Ey)}
        f = oracle.make_field(spec)
        G = _photons(1, eps, (1.0, 0.0, 0.0))
        dt, N = 0.05, 400
        sim = oracle.Sim(dt=dt, procs=oracle.PROC_VB, seed=1, next_id=1)
        for s in range(N):
            sim.photon_step(f, G, None, None, s)
        chi = XI_L * eps * 2 * Ey
        M = oracle.tables().vb_M(chi)
        dphi = (M[0] - M[1]) * ALPHA / (90 * math.pi) * chi * chi * dt / (eps * XI_L)
        assert G.xi1[0] == pytest.approx(math.cos(N * dphi), abs=1e-12)
        assert G.xi2[0] == pytest.approx(math.sin(N * dphi), abs=1e-12)
        assert G.xi3[0] == 0.0
        assert G.x[0] == pytest.approx(N * dt, rel=1e-14)
        if label == "low":
            D = ALPHA / (90 * math.pi) * chi * chi / eps ** 2
            ref = GOLD["vb_low_chi_phase_factor"]["value"] * D * (eps / XI_L) * dt
            assert dphi == pytest.approx(ref, rel=1e-6)


def test_frame_rotation_algebra():
    """A photon whose stored basis is rotated by psi against E_red: ROT(psi) keeps |xi|,
    maps a pure state polarised along the old e1 to the state polarised along the same
    physical direction in the new basis, and two successive changes compose."""
    eps = 50.0
    spec = {"kind": oracle.FIELD_CONST, "e0": (0, 0.3, 0.0), "b0": (0, 0, -0.3)}   # E_red along y
    f = oracle.make_field(spec)
    for psi in (0.3, 1.1, math.pi / 2, math.pi):
        e1 = (0, math.cos(psi), -math.sin(psi))     # new e1 (= y) = cos(psi) e1 + sin(psi) e2, e2 = x cross e1
        G = _photons(1, eps, (0.0, 0.0, 1.0), e1=e1)   # linear along old e1
        sim = oracle.Sim(dt=1e-9, procs=oracle.PROC_VB, seed=1, next_id=1)
        sim.photon_step(f, G, None, None, 0)
        xi = np.array([G.xi1[0], G.xi2[0], G.xi3[0]])
        assert np.linalg.norm(xi) == pytest.approx(1.0, abs=1e-12)
        # linear polarisation at angle -psi from the new e1: xi3 = cos(2psi), xi1 = -sin(2psi)
        assert xi[2] == pytest.approx(math.cos(2 * psi), abs=1e-9)
        assert xi[0] == pytest.approx(-math.sin(2 * psi), abs=1e-9)
        assert np.allclose([G.e1x[0], G.e1y[0], G.e1z[0]], [0, 1, 0], atol=1e-15)


def test_nbw_events():
    """Pair events: energy shared exactly, momenta along the photon, pairs appended in
    photon order with consecutive ids (electron, positron), photon removed; the event
    fraction equals W dt; the positron mean spin along its SQA follows |D|/C."""
    eps, chi, n = 4000.0, 2.0, 200_000
    Ey = chi / (XI_L * eps * 2)
    spec = {"kind": oracle.FIELD_CONST, "e0": (0, Ey, 0), "b0": (0, 0, -Ey)}
    f = oracle.make_field(spec)
    G = _photons(n, eps, (0.0, 0.0, 0.4))
    Ja, Jb = oracle.nbw_Ja(chi), oracle.nbw_Jb(chi)
    W = ALPHA / (SQ3 * math.pi * XI_L * eps) * (Ja - 0.4 * Jb)
    dt = 0.03 / W
    em, ep = oracle.LeptonArrays.empty(n, -1), oracle.LeptonArrays.empty(n, 1)
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NBW, seed=4, next_id=500)
    sim.photon_step(f, G, em, ep, 9)
    m = em.count
    assert ep.count == m
    assert abs(m - 0.03 * n) < 4.5 * math.sqrt(n * 0.03)
    dead = np.where(G.alive[:n] == 0)[0]
    assert len(dead) == m
    assert np.array_equal(em.id[:m], 500 + 2 * np.arange(m, dtype=np.uint64))
    assert np.array_equal(ep.id[:m], 501 + 2 * np.arange(m, dtype=np.uint64))
    e_m = np.sqrt(1 + em.px[:m] ** 2 + em.py[:m] ** 2 + em.pz[:m] ** 2)
    e_p = np.sqrt(1 + ep.px[:m] ** 2 + ep.py[:m] ** 2 + ep.pz[:m] ** 2)
    assert np.allclose(e_m + e_p, eps, rtol=1e-12)
    assert np.allclose(em.py[:m], 0) and np.allclose(ep.pz[:m], 0)
    Sm = np.stack([em.sx[:m], em.sy[:m], em.sz[:m]])
    Sp = np.stack([ep.sx[:m], ep.sy[:m], ep.sz[:m]])
    assert np.allclose(np.linalg.norm(Sm, axis=0), 1, atol=1e-12)
    assert np.allclose(np.linalg.norm(Sp, axis=0), 1, atol=1e-12)
    # survivors moved by dt along x; the dead did not
    alive = G.alive[:n] == 1
    assert np.allclose(G.x[:n][alive], dt) and np.all(G.x[:n][~alive] == 0)
    # energy spectrum symmetric about 1/2 for linear (xi2 = 0) photons: mean delta = 1/2
    d = e_p / eps
    assert abs(d.mean() - 0.5) < 4.5 * d.std() / math.sqrt(m)
    # positron polarisation along b = n x a (= z): <S+.z> = E[D_z / C] over the spectrum
    rho = lambda dd: 2 / (3 * chi * dd * (1 - dd))
    import scipy.special as sp
    num = den = 0.0
    for dd in np.linspace(1e-3, 1 - 1e-3, 2001):
        r = rho(dd)
        K1, K2, I = sp.kv(1 / 3, r), sp.kv(2 / 3, r), oracle.int_bessel_k(1 / 3, r)
        Cc = I + (dd * dd + (1 - dd) ** 2) / (dd * (1 - dd)) * K2 - 0.4 * K2
        Dz = -(1 / dd - 0.4 / (1 - dd)) * K1
        num += Dz
        den += Cc
    assert abs(Sp[2].mean() - num / den) < 4.5 * Sp[2].std() / math.sqrt(m) + 2e-3


def test_compaction_is_stable():
    G = _photons(10, 10.0, (0, 0, 0))
    G.alive[[1, 4, 5, 9]] = 0
    G.x[:10] = np.arange(10)
    sim = oracle.Sim(dt=0.1, procs=0, seed=1, next_id=1)
    assert sim.compact(G) == 6
    assert np.array_equal(G.x[:6], [0, 2, 3, 6, 7, 8])
    assert np.array_equal(G.id[:6], np.array([0, 2, 3, 6, 7, 8], np.uint64))


@pytest.mark.slow
def test_sokolov_ternov_buildup():
    """Storage-ring stand-in: electrons in a uniform B at fixed chi, |p| restored to gamma0
    after every step by the harness.  <S.B_hat> -> -P_inf (1 - exp(-t/tau)) with
    P_inf = psi3/psi1 and 1/tau = alpha psi1/(sqrt3 pi xi_L gamma) (Sec. I, III.B.2)."""
    gamma, chi, n = 1000.0, 1.0, 20_000
    pm = math.sqrt(gamma * gamma - 1)
    B = chi / (XI_L * pm)
    f = oracle.make_field({"kind": oracle.FIELD_CONST, "e0": (0, 0, 0), "b0": (0, 0, B)})
    rng = np.random.default_rng(1)
    S = rng.normal(size=(3, n)); S /= np.linalg.norm(S, axis=0)
    ph = rng.uniform(0, 2 * math.pi, n)
    st = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "px": pm * np.cos(ph), "py": pm * np.sin(ph),
          "pz": np.zeros(n), "w": np.ones(n), "sx": S[0], "sy": S[1], "sz": S[2],
          "id": np.arange(n, dtype=np.uint64)}
    L = oracle.LeptonArrays.from_state(st, charge=-1)
    psi = oracle.rbmt_psi(chi)
    C = ALPHA / (SQ3 * math.pi * XI_L * gamma)
    rate = C * psi[0]
    dt = 0.02 / (C * oracle.ncs_Ia(chi))
    steps = int(round(1.0 / (rate * dt)))      # one build-up time
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS, seed=3, next_id=1 << 40)
    for s in range(steps):
        E6 = np.zeros(6 * n)
        sim.push_spin(f, L, s, E6)
        sim.emit(L, E6, None, s)
        p = np.stack([L.px[:n], L.py[:n], L.pz[:n]])
        p *= pm / np.linalg.norm(p, axis=0)
        L.px[:n], L.py[:n], L.pz[:n] = p
    sB = L.sz[:n]
    expect = -(psi[2] / psi[0]) * (1 - math.exp(-steps * dt * rate))
    assert abs(sB.mean() - expect) < 4.5 * sB.std() / math.sqrt(n) + 0.01 * abs(expect), (sB.mean(), expect)

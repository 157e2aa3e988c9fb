"""Oracle pins of the radiative-correction stage (Sec. III.A: Landau-Lifshitz force and its
quantum-corrected form; Sec. III.B: radiative T-BMT), against identities and closed forms
that do not come from the oracle's own formulas:

  * the RAD table (g, psi1..3 on the NCS rate grid) interpolates the direct quadratures,
    whose small-chi limits are pinned in test_oracle_rates;
  * the force: in a pure magnetic field beta.F equals minus the Larmor power
    (2/3)(alpha/xi_L) chi^2 for any momentum; it vanishes for motion along a pure electric
    field (hyperbolic motion radiates no reaction force), which fixes the 1/gamma of the
    E(p.E) term; the third term alone is -(2/3)(alpha/xi_L) chi^2 beta;
  * synchrotron cooling in a uniform B: dgamma/dt = -K (gamma^2 - 1), K = (2/3) alpha xi_L B^2,
    solved by gamma(t) = coth(K t + arcoth gamma0); the scheme converges at first order;
  * radiative T-BMT in a uniform B with S along B: S.B + psi3/psi1 decays by exactly
    (1 - P psi1 dt/2)^2 per step (two half kicks around a rotation that leaves S fixed);
  * mode 0 is the plain push (bitwise).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

SQ3 = math.sqrt(3.0)
A, XI = oracle.ALPHA, oracle.XI_L


def test_rad_table_interpolates_the_quadratures():
    """Table against direct quadrature at off-node chi (the spec's bound for FP64 tables is
    1e-6; this one interpolates flat functions and stays near 1e-8)."""
    T = oracle.tables()
    for chi in np.geomspace(1.3e-5, 900.0, 37):
        g, p1, p2, p3 = T.rad(chi)
        ref = oracle.rbmt_psi(chi)
        assert g == pytest.approx(oracle.ncs_power_ratio(chi), rel=1e-7)
        for k, v in enumerate((p1, p2, p3)):
            assert abs(v - ref[k]) < 1e-7 * abs(ref[0]), (chi, k, v, ref[k])
    # below the grid: first-order Gaunt factor and chi^3 scaling of the psi integrals
    c = 3e-7
    g, p1, _, p3 = T.rad(c)
    assert g == 1 - 55 * SQ3 / 16 * c
    assert p3 / p1 == pytest.approx(8 / (5 * SQ3), abs=3e-5)
    assert p1 / c ** 3 == pytest.approx(15 * math.pi / 8, rel=2e-5)


def test_ll_force_pure_magnetic_field_is_the_larmor_loss():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rng.normal(size=3) * 10 ** rng.uniform(0, 4)
        B = rng.normal(size=3) * 10 ** rng.uniform(-1, 2)
        g = math.sqrt(1 + p @ p)
        F = oracle.ll_force(g, p, [0, 0, 0], B)
        chi = XI * np.linalg.norm(np.cross(p, B))
        assert (p / g) @ F == pytest.approx(-2 / 3 * A / XI * chi ** 2, rel=1e-12)


def test_ll_force_vanishes_along_a_pure_electric_field():
    rng = np.random.default_rng(2)
    for _ in range(10):
        E = rng.normal(size=3) * 30
        p = E / np.linalg.norm(E) * 10 ** rng.uniform(0, 4)
        g = math.sqrt(1 + p @ p)
        F = oracle.ll_force(g, p, E, [0, 0, 0])
        scale = 2 / 3 * A * XI * (E @ E) * np.linalg.norm(p) / g   # size of either cancelling term
        # E^2 - (beta.E)^2 = E^2/gamma^2 is formed by cancellation: rounding ~ eps gamma^2
        assert np.linalg.norm(F) < (1e-13 + 4e-16 * g * g) * scale


def test_ll_force_third_term_and_head_on_limit():
    """Head-on with a crossed field (E = E0 y, B = -E0 z: a wave along -x), p = gamma beta x:
    the force is -(2/3)(alpha/xi_L) chi^2 beta up to terms smaller by 1/gamma^2, with
    chi = xi_L gamma (1 + beta) E0."""
    E0 = 50.0
    for gam in (1e3, 1e4):
        p = np.array([math.sqrt(gam * gam - 1), 0, 0])
        F = oracle.ll_force(gam, p, [0, E0, 0], [0, 0, -E0])
        beta = p / gam
        chi = XI * gam * (1 + beta[0]) * E0
        ref = -2 / 3 * A / XI * chi ** 2 * beta
        assert F[0] == pytest.approx(ref[0], rel=3 / gam ** 2)
        assert abs(F[1]) < 3 / gam ** 2 * abs(ref[0])


def _lepton(p, S):
    st = {k: np.zeros(1) for k in ("x", "y", "z", "px", "py", "pz", "sx", "sy", "sz")}
    st["px"][:], st["py"][:], st["pz"][:] = p
    st["sx"][:], st["sy"][:], st["sz"][:] = S
    st["w"] = np.ones(1)
    st["id"] = np.zeros(1, np.uint64)
    return oracle.LeptonArrays.from_state(st, charge=-1)


def _cool(gamma0, B, t_end, nsteps, mode):
    dt = t_end / nsteps
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS, seed=1, next_id=0)
    field = oracle.make_field({"kind": W.FIELD_CONST, "e0": (0, 0, 0), "b0": (0, 0, B)})
    L = _lepton([math.sqrt(gamma0 ** 2 - 1), 0, 0], [0, 0, 1])
    for s in range(nsteps):
        sim.push_radiative(field, L, s, mode)
    p = np.array([L.px[0], L.py[0], L.pz[0]])
    return math.sqrt(1 + p @ p), p


def test_synchrotron_cooling_closed_form_first_order():
    gamma0, B, t_end = 1e4, 100.0, 2.0
    K = 2 / 3 * A * XI * B * B
    exact = 1 / math.tanh(K * t_end + math.atanh(1 / gamma0))
    assert gamma0 / exact > 2.5          # strong cooling over the run
    errs = []
    for n in (800, 1600, 3200):
        g, p = _cool(gamma0, B, t_end, n, oracle.RR_LL)
        assert abs(p[2]) < 1e-12 * g     # stays in the plane
        errs.append(abs(g / exact - 1))
    assert errs[-1] < 5e-3
    for a, b in zip(errs[:-1], errs[1:]):
        assert 1.8 < a / b < 2.2         # first order in dt


def test_quantum_corrected_cooling_follows_the_gaunt_factor():
    """MLL: dgamma/dt = -K p^2 g(xi_L p B); reference from a fine RK4 integration with the
    power ratio from direct quadrature; the scheme converges to it at first order."""
    gamma0, B, t_end = 3e4, 800.0, 0.05
    K = 2 / 3 * A * XI * B * B

    def rate(gm):
        pp = gm * gm - 1
        return -K * pp * oracle.ncs_power_ratio(XI * math.sqrt(pp) * B)

    gm, n = gamma0, 4000
    h = t_end / n
    for _ in range(n):
        k1 = rate(gm); k2 = rate(gm + h / 2 * k1); k3 = rate(gm + h / 2 * k2); k4 = rate(gm + h * k3)
        gm += h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    g_ll, _ = _cool(gamma0, B, t_end, 1000, oracle.RR_LL)
    errs = []
    for steps in (1000, 2000):
        g, _ = _cool(gamma0, B, t_end, steps, oracle.RR_MLL)
        errs.append(abs(g / gm - 1))
    assert g_ll < 0.8 * gm               # the quantum correction matters here (chi ~ 0.06-0.1)
    assert errs[-1] < 2e-3 and 1.7 < errs[0] / errs[1] < 2.3


@pytest.mark.parametrize("s0", [1.0, 0.3, -0.5])
def test_radiative_tbmt_decay_is_exact_for_the_discrete_scheme(s0):
    gamma0, B, dt, n = 5e3, 200.0, 2 * math.pi / 500, 400
    sim = oracle.Sim(dt=dt, procs=oracle.PROC_NCS, seed=1, next_id=0)
    field = oracle.make_field({"kind": W.FIELD_CONST, "e0": (0, 0, 0), "b0": (0, 0, B)})
    pmag = math.sqrt(gamma0 ** 2 - 1)
    L = _lepton([pmag, 0, 0], [0, 0, s0])
    for s in range(n):
        sim.push_radiative(field, L, s, oracle.RR_RBMT)
    # time-centred chi of a Boris step in a pure B: |beta^n| = |beta| / sqrt(1 + tau^2)
    tau = dt * B / (2 * gamma0)
    chi = XI * pmag * B / math.sqrt(1 + tau * tau)
    psi = oracle.rbmt_psi(chi)
    lam = A / (SQ3 * math.pi * XI * gamma0) * psi[0]
    c = psi[2] / psi[0]                  # electron: fixed point S = -(psi3/psi1) B^
    want = -c + (1 - lam * dt / 2) ** (2 * n) * (s0 + c)
    assert L.sz[0] == pytest.approx(want, rel=2e-7)
    assert abs(L.sx[0]) < 1e-14 and abs(L.sy[0]) < 1e-14
    assert math.sqrt(1 + L.px[0] ** 2 + L.py[0] ** 2) == pytest.approx(gamma0, rel=1e-14)   # no force
    assert (1 - lam * dt / 2) ** (2 * n) < 0.9   # the spin moved noticeably


def test_mode_zero_is_the_plain_push():
    cfg = W.c1(300)
    field = oracle.make_field(cfg["field"])
    a = oracle.LeptonArrays.from_state(cfg["leptons"])
    b = oracle.LeptonArrays.from_state(cfg["leptons"])
    s1 = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=1, next_id=0)
    s2 = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=1, next_id=0)
    for s in range(700, 760):
        s1.push_spin(field, a, s)
        s2.push_radiative(field, b, s, 0)
    for k in ("x", "y", "z", "px", "py", "pz", "sx", "sy", "sz"):
        assert np.array_equal(getattr(a, k)[:a.count], getattr(b, k)[:b.count])


def test_radiation_reaction_in_the_plane_wave_workload():
    """The plane-wave workload with LL, MLL and radiative spin: electrons lose energy
    (MLL less than LL), spins stay at most unit length, nothing is flagged."""
    cfg = W.c1(200)
    cfg["leptons"]["px"] *= 4.0
    field = oracle.make_field(dict(cfg["field"], a0=100.0))
    out = {}
    for mode in (0, oracle.RR_LL, oracle.RR_MLL | oracle.RR_RBMT):
        L = oracle.LeptonArrays.from_state(cfg["leptons"])
        sim = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=1, next_id=0)
        for s in range(0, 1600):
            sim.push_radiative(field, L, s, mode)
        out[mode] = np.sqrt(1 + L.px ** 2 + L.py ** 2 + L.pz ** 2).mean()
        assert sim.status == 0
        assert np.all(np.sqrt(L.sx ** 2 + L.sy ** 2 + L.sz ** 2) <= 1 + 1e-12)
    e0, e_ll, e_mll = out[0], out[oracle.RR_LL], out[oracle.RR_MLL | oracle.RR_RBMT]
    assert e_ll < 0.98 * e0 and e_ll < e_mll < e0

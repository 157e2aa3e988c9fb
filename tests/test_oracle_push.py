"""Pins of the oracle's fields, Boris pusher, T-BMT rotation and chi: closed forms and the
invariants of motion in a plane wave (Sec. II.A, III.A.3, III.B.3)."""
import math

import numpy as np
import pytest

import oracle
from oracle import A_E, XI_L

TWO_PI = 2 * math.pi


def test_boris_pure_magnetic_rotation():
    """Pure B: |p| exact to rounding and rotation angle 2 atan(|tau|) per step."""
    B = np.array([0.3, -1.2, 40.0])
    p = np.array([100.0, 30.0, -7.0])
    dt = 0.05
    for q in (-1.0, 1.0):
        p1, pm, pp = oracle.boris(q, dt, np.zeros(3), B, p)
        assert np.linalg.norm(p1) == pytest.approx(np.linalg.norm(p), rel=1e-15)
        g = math.sqrt(1 + p @ p)
        tau = 0.5 * q * dt * B / g
        bh = B / np.linalg.norm(B)
        a, b = p - bh * (p @ bh), p1 - bh * (p1 @ bh)
        ang = math.atan2(np.linalg.norm(np.cross(a, b)), a @ b)
        assert ang == pytest.approx(2 * math.atan(np.linalg.norm(tau)), rel=1e-12)
        # the sense of rotation follows dp/dt = q p x B / gamma
        assert np.sign(np.cross(a, b) @ bh) == np.sign(-q)


def test_boris_uniform_electric_field():
    """Pure E along x: p_x grows by q E dt exactly each step."""
    p = np.array([0.0, 0.0, 0.0])
    for k in range(100):
        p, _, _ = oracle.boris(-1.0, 0.1, np.array([2.0, 0, 0]), np.zeros(3), p)
    assert p[0] == pytest.approx(-20.0, rel=1e-14)


def _pw_run(dt, tend, a0=5.0):
    """Electron (initially at rest) in the LP plane wave; returns final p and A(phi)."""
    spec = {"kind": oracle.FIELD_PW, "circular": 0, "a0": a0, "ncycles": 4.0, "phase0": 0.0,
            "pol_angle": 0.0, "phi_start": 0.0}
    f = oracle.make_field(spec)
    L = oracle.LeptonArrays.from_state({"x": np.array([-1.0]), "y": np.zeros(1), "z": np.zeros(1),
                                        "px": np.array([0.0]), "py": np.zeros(1), "pz": np.zeros(1),
                                        "w": np.ones(1), "sx": np.zeros(1), "sy": np.ones(1), "sz": np.zeros(1),
                                        "id": np.zeros(1, np.uint64)}, charge=-1)
    sim = oracle.Sim(dt=dt, procs=0, seed=1, next_id=10)
    n = int(round(tend / dt))
    traj = []
    for s in range(n):
        sim.push_spin(f, L, s)
        traj.append((L.x[0], L.px[0], L.py[0], L.pz[0]))
    return np.array(traj), spec, n


def _A(phi, spec):
    L = TWO_PI * spec["ncycles"]
    if phi < 0 or phi > L:
        return 0.0
    return spec["a0"] * math.sin(math.pi * phi / L) ** 2 * math.sin(phi)


def test_plane_wave_invariants_second_order():
    """In a plane wave along -x (phase t + x), the transverse canonical momentum
    p_y + q A_y and the light-front energy gamma - (-x_hat).p = gamma + p_x are conserved
    (analytic solution of Sec. III.A.3, with the proper-time label read as the phase).
    The Boris error in them shrinks as dt^2."""
    errs = []
    for dt in (0.04, 0.02, 0.01):
        traj, spec, n = _pw_run(dt, 30.0)
        e1 = e2 = 0.0
        for s in range(n):
            x, px, py, pz = traj[s]
            # x is at t = (s+1) dt, p at t = (s+1/2) dt: evaluate A at the half step phase
            xh = x - 0.5 * dt * px / math.sqrt(1 + px * px + py * py + pz * pz)
            phi = (s + 0.5) * dt + xh
            e1 = max(e1, abs(py - _A(phi, spec)))      # q = -1: p_y - A_y = 0
            g = math.sqrt(1 + px * px + py * py + pz * pz)
            e2 = max(e2, abs(g + px - 1.0))
        errs.append((e1, e2))
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 1.8), (errs, order)
    assert errs[-1, 0] < 1e-2 and errs[-1, 1] < 1e-2


def test_pw_field_is_minus_dA_dphi():
    spec = {"kind": oracle.FIELD_PW, "circular": 1, "a0": 3.0, "ncycles": 2.0, "phase0": 0.4,
            "pol_angle": 0.3, "phi_start": 1.0}
    L = TWO_PI * spec["ncycles"]

    def A(phi):
        p = phi - spec["phi_start"]
        if p < 0 or p > L:
            return np.zeros(3)
        env = math.sin(math.pi * p / L) ** 2
        c, s = math.cos(spec["pol_angle"]), math.sin(spec["pol_angle"])
        e1, e2 = np.array([0, c, s]), np.array([0, -s, c])
        return spec["a0"] * env * (math.sin(p + spec["phase0"]) * e1 + math.cos(p + spec["phase0"]) * e2)
    h = 1e-5
    for phi in (2.0, 5.5, 9.0, 13.0):
        t, x = phi - 0.7, 0.7
        E, B = oracle.field_eval(spec, t, [x, 0.2, -0.4])
        dA = (A(phi + h) - A(phi - h)) / (2 * h)
        assert np.allclose(E, -dA, atol=1e-8)
        assert np.allclose(B, np.cross([-1, 0, 0], E), atol=1e-15)


def test_gaussian_focus_profile():
    """At the focus on axis, the CP focused pulse has |E| = a0 env, E perpendicular to x,
    B = -x_hat cross E; off axis it falls as exp(-r^2/w0^2); beyond z_R it falls as
    1/sqrt(1+(x/z_R)^2)."""
    w0 = 3 * TWO_PI
    spec = {"kind": oracle.FIELD_GAUSS, "circular": 1, "a0": 100.0, "ncycles": 10.0, "phase0": 0.0,
            "pol_angle": 0.0, "w0": w0, "x_focus": 0.0, "phi_start": 0.0}
    t = 10 * math.pi       # envelope centre at x = 0
    E, B = oracle.field_eval(spec, t, [0.0, 0.0, 0.0])
    assert np.linalg.norm(E) == pytest.approx(100.0, rel=1e-14)
    assert E[0] == 0 and np.allclose(B, np.cross([-1, 0, 0], E))
    r = 0.7 * w0
    E2, _ = oracle.field_eval(spec, t, [0.0, r, 0.0])
    assert np.linalg.norm(E2) == pytest.approx(100.0 * math.exp(-(r / w0) ** 2), rel=1e-13)
    zr = 0.5 * w0 * w0
    E3, _ = oracle.field_eval(spec, t - 2 * zr, [2 * zr, 0.0, 0.0])
    assert np.linalg.norm(E3) == pytest.approx(100.0 / math.sqrt(5.0), rel=1e-13)


def _grid_spec(fill):
    nx, ny, dx, dy, x0, y0 = 24, 20, 0.3, 0.25, -3.0, -2.0
    comps = []
    for c, (hx, hy) in enumerate([(1, 0), (0, 1), (0, 0), (0, 1), (1, 0), (1, 1)]):
        X = x0 + dx * (np.arange(nx) + 0.5 * hx)
        Y = y0 + dy * (np.arange(ny) + 0.5 * hy)
        comps.append(fill(c, X[None, :], Y[:, None]).astype(np.float32))
    return {"kind": oracle.FIELD_GRID2D, "grid": comps, "nx": nx, "ny": ny, "dx": dx, "dy": dy,
            "gx0": x0, "gy0": y0}


def test_grid_tsc_reproduces_constant_and_linear_fields():
    """TSC weights sum to one and reproduce linear functions exactly on the staggered
    Yee positions (Sec. II.D-E with the squared side weights)."""
    const = _grid_spec(lambda c, X, Y: np.full(np.broadcast(X, Y).shape, 1.5 + c))
    lin = _grid_spec(lambda c, X, Y: 0.5 * X - 0.25 * Y + c + 0 * X * Y)
    rng = np.random.default_rng(3)
    for _ in range(50):
        r = [rng.uniform(-2.0, 3.0), rng.uniform(-1.2, 2.0), 0.0]
        E, B = oracle.field_eval(const, 0.0, r)
        assert np.allclose(np.r_[E, B], 1.5 + np.arange(6), rtol=1e-6)
        E, B = oracle.field_eval(lin, 0.0, r)
        assert np.allclose(np.r_[E, B], 0.5 * r[0] - 0.25 * r[1] + np.arange(6), atol=2e-6)


def test_chi_closed_forms():
    # pure magnetic field: chi = xi_L |p x B|
    p, B = np.array([800.0, 20.0, 0.0]), np.array([0.0, 0.0, 50.0])
    assert oracle.chi_e(p, np.zeros(3), B) == pytest.approx(XI_L * np.linalg.norm(np.cross(p, B)), rel=1e-14)
    # head-on plane wave: chi = xi_L gamma (1 + beta) |E|
    g = 1000.0
    p = np.array([math.sqrt(g * g - 1), 0.0, 0.0])
    E, B = np.array([0.0, 30.0, 0.0]), np.array([0.0, 0.0, -30.0])
    beta = p[0] / g
    assert oracle.chi_e(p, E, B) == pytest.approx(XI_L * g * (1 + beta) * 30.0, rel=1e-13)
    # co-propagating: chi = xi_L gamma (1 - beta)|E| -> tiny
    assert oracle.chi_e(-p, E, B) == pytest.approx(XI_L * g * (1 - beta) * 30.0, rel=1e-6)
    # photons
    k = np.array([500.0, 0, 0])
    assert oracle.chi_gamma(k, E, B) == pytest.approx(XI_L * 500 * 60.0, rel=1e-14)
    assert oracle.chi_gamma(-k, E, B) == pytest.approx(0.0, abs=1e-12)


def test_bmt_uniform_magnetic_field():
    """T-BMT rotation in a uniform B with beta perpendicular to B: the spin turns about B
    by 2 atan(|t|) per step, t = (q dt/2)(a_e + 1/gamma) B; |S| stays 1; relative to p the
    spin precesses by the anomalous part only.  With a_e = 0 the helicity S.p is exactly
    that of the momentum rotation (S locked to p)."""
    B = np.array([0.0, 0.0, 25.0])
    p = np.array([300.0, 0.0, 0.0])
    S = np.array([0.6, 0.8, 0.0])
    dt = 0.02
    for q in (-1.0, 1.0):
        p1, pm, pp = oracle.boris(q, dt, np.zeros(3), B, p)
        S1 = oracle.bmt(q, A_E, dt, np.zeros(3), B, pm, pp, S)
        g = math.sqrt(1 + pm @ pm)
        tnorm = abs(0.5 * q * dt * (A_E + 1 / g) * B[2])
        ang = math.atan2(S[0] * S1[1] - S[1] * S1[0], S @ S1)
        assert abs(ang) == pytest.approx(2 * math.atan(tnorm), rel=1e-12)
        assert np.linalg.norm(S1) == pytest.approx(1.0, abs=1e-15)
        S0 = oracle.bmt(q, 0.0, dt, np.zeros(3), B, pm, pp, S)
        assert S0 @ p1 / np.linalg.norm(p1) == pytest.approx(S @ p / np.linalg.norm(p), abs=1e-12)


def test_bmt_spin_locked_to_momentum_in_electric_field():
    """g = 2 (a_e = 0): for a particle moving perpendicular to a pure E the spin rotates
    with 1/(gamma+1) times beta x E; S.beta is not conserved but |S| = 1 (pure rotation)."""
    E = np.array([0.0, 10.0, 0.0])
    p = np.array([50.0, 0.0, 0.0])
    S = np.array([0.0, 0.0, 1.0])
    p1, pm, pp = oracle.boris(-1.0, 0.01, E, np.zeros(3), p)
    S1 = oracle.bmt(-1.0, 0.0, 0.01, E, np.zeros(3), pm, pp, S)
    assert np.linalg.norm(S1) == pytest.approx(1.0, abs=1e-15)
    assert S1 == pytest.approx(S, abs=1e-12)   # rotation axis beta x E is along z = S

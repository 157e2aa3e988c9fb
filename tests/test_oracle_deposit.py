"""Pins of the current-deposition oracle (Sec. II.C, charge conservation; TSC shapes of
Sec. II.E) against properties that do not come from its own formulas:

  * the discrete continuity equation (rho1 - rho0)/dt + div J = 0 at every node, rho from
    the TSC charge assignment of the start and end positions (the defining property);
  * total current: sum J dx dy = sum Q v for each component (TSC keeps the first moment);
  * a straight move along x: the charge through face i+1/2 is the mass of the triangular
    charge cloud (whose cell integrals are the TSC weights) that crossed the face, from the
    cloud's cumulative distribution;
  * Jz is the step average of the product of the linearly interpolated shapes: two-point
    Gauss-Legendre of that product (exact for a quadratic in t); a move along z only
    gives Q vz S_x S_y and no in-plane current; a particle at rest deposits nothing;
  * Gauss's law with the field solver: div E - rho stays at its initial value to rounding
    over many steps of moving particles (the paper's argument for solving only the curl
    equations).
"""
import math

import numpy as np
import pytest

from oracle import deposit as D
from oracle import yee

NX, NY, DX, DY = 40, 24, 0.21, 0.17


def _particles(n, seed, frac=0.95, gx0=0.0, gy0=0.0):
    rng = np.random.default_rng(seed)
    xa = gx0 + rng.uniform(-2 * DX, (NX + 2) * DX, n)       # some outside the box (periodic)
    ya = gy0 + rng.uniform(-2 * DY, (NY + 2) * DY, n)
    za = rng.normal(0, 1, n)
    xb = xa + rng.uniform(-frac, frac, n) * DX
    yb = ya + rng.uniform(-frac, frac, n) * DY
    zb = za + rng.uniform(-0.1, 0.1, n)
    w = rng.uniform(0.5, 2.0, n)
    return xa, ya, za, xb, yb, zb, w


@pytest.mark.parametrize("q,gx0,gy0", [(-1, 0.0, 0.0), (1, -3.3, 0.7)])
def test_continuity_equation_holds_node_by_node(q, gx0, gy0):
    dt, qs = 0.05, 0.3
    xa, ya, za, xb, yb, zb, w = _particles(3000, 1, gx0=gx0, gy0=gy0)
    Jx, Jy, Jz = D.deposit(xa, ya, za, xb, yb, zb, w, q, qs, dt, NX, NY, DX, DY, gx0, gy0)
    r0 = D.rho(xa, ya, w, q, qs, NX, NY, DX, DY, gx0, gy0)
    r1 = D.rho(xb, yb, w, q, qs, NX, NY, DX, DY, gx0, gy0)
    res = (r1 - r0) / dt + D.divergence(Jx, Jy, DX, DY)
    scale = np.abs(r0).max() / dt
    assert np.abs(res).max() < 1e-12 * scale
    assert np.abs(r1 - r0).max() > 0.01 * np.abs(r0).max()          # the charge really moved
    # total charge is kept
    assert r1.sum() == pytest.approx(r0.sum(), rel=1e-12)
    assert r0.sum() * DX * DY == pytest.approx(q * qs * w.sum(), rel=1e-12)


def test_total_current_is_charge_times_velocity():
    dt, q, qs = 0.07, -1, 1.7
    xa, ya, za, xb, yb, zb, w = _particles(2000, 2)
    Jx, Jy, Jz = D.deposit(xa, ya, za, xb, yb, zb, w, q, qs, dt, NX, NY, DX, DY)
    Q = q * qs * w
    for J, d in ((Jx, xb - xa), (Jy, yb - ya), (Jz, zb - za)):
        assert J.sum() * DX * DY == pytest.approx((Q * d / dt).sum(), rel=1e-11, abs=1e-12 * np.abs(Q).sum() / dt)


def _cloud_cdf(u):
    """mass of the unit triangular cloud T(s) = max(0, 1 - |s|) below s = u"""
    if u <= -1:
        return 0.0
    if u <= 0:
        return 0.5 * (1 + u) ** 2
    if u <= 1:
        return 1 - 0.5 * (1 - u) ** 2
    return 1.0


def test_move_along_x_is_the_cloud_flux_through_each_face():
    dt, q, qs = 0.1, 1, 1.0
    for Xa, Xb in ((5.2, 5.9), (7.45, 7.55), (10.6, 9.8), (3.0, 3.0 + 0.999)):
        Ya = 11.3
        Jx, Jy, Jz = D.deposit([Xa * DX], [Ya * DY], [0.0], [Xb * DX], [Ya * DY], [0.0], [1.0], q, qs, dt,
                               NX, NY, DX, DY)
        assert np.all(Jy == 0) and np.all(Jz == 0)
        jy, wy = D.tsc_weights(Ya)
        for i in range(NX):
            face = i + 0.5
            crossed = _cloud_cdf(face - Xa) - _cloud_cdf(face - Xb)      # mass moved past the face
            for k in range(3):
                want = crossed * wy[k] / (DY * dt)
                assert Jx[jy - 1 + k, i] == pytest.approx(want, abs=1e-13 / (DY * dt)), (Xa, Xb, i)
        assert np.count_nonzero(Jx) >= 3


def test_jz_is_the_step_average_of_the_interpolated_shapes():
    dt, q, qs = 0.05, -1, 2.0
    g = (0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3))
    rng = np.random.default_rng(5)
    for _ in range(20):
        Xa, Ya = rng.uniform(5, 30), rng.uniform(5, 18)
        Xb, Yb = Xa + rng.uniform(-0.9, 0.9), Ya + rng.uniform(-0.9, 0.9)
        za, zb = 0.3, 0.3 + rng.uniform(-0.05, 0.05)
        _, _, Jz = D.deposit([Xa * DX], [Ya * DY], [za], [Xb * DX], [Yb * DY], [zb], [1.0], q, qs, dt,
                             NX, NY, DX, DY)
        # shapes on absolute node indices, linearly interpolated in t
        want = np.zeros((NY, NX))
        for t in g:
            sx = np.zeros(NX); sy = np.zeros(NY)
            for X, s, f in ((Xa, sx, 1 - t), (Xb, sx, t)):
                j, ws = D.tsc_weights(X)
                for k in range(3):
                    s[j - 1 + k] += f * ws[k]
            for Y, s, f in ((Ya, sy, 1 - t), (Yb, sy, t)):
                j, ws = D.tsc_weights(Y)
                for k in range(3):
                    s[j - 1 + k] += f * ws[k]
            want += 0.5 * np.outer(sy, sx)
        want *= q * qs * (zb - za) / dt / (DX * DY)
        assert np.abs(Jz - want).max() < 1e-13 * np.abs(want).max()


def test_move_along_z_only_and_rest():
    dt = 0.05
    Jx, Jy, Jz = D.deposit([2.31], [1.77], [0.0], [2.31], [1.77], [0.04], [1.5], -1, 1.0, dt, NX, NY, DX, DY)
    assert np.all(Jx == 0) and np.all(Jy == 0)
    r = D.rho([2.31], [1.77], [1.5], -1, 1.0, NX, NY, DX, DY)
    assert np.allclose(Jz, r * 0.04 / dt, rtol=1e-14, atol=0)
    Jx, Jy, Jz = D.deposit([2.31], [1.77], [0.5], [2.31], [1.77], [0.5], [1.5], -1, 1.0, dt, NX, NY, DX, DY)
    assert not Jx.any() and not Jy.any() and not Jz.any()


def test_displacement_of_a_cell_is_refused():
    with pytest.raises(ValueError):
        D.deposit([1.0], [1.0], [0.0], [1.0 + DX], [1.0], [0.0], [1.0], -1, 1.0, 0.1, NX, NY, DX, DY)


def test_gauss_law_is_kept_by_the_solver_with_the_deposited_current():
    """Particles on straight lines at |v| < 1, the solver advancing E with their current:
    div E - rho keeps its initial value at every node."""
    rng = np.random.default_rng(9)
    n, steps = 400, 60
    dt = 0.6 / math.sqrt(1 / DX ** 2 + 1 / DY ** 2)
    x = rng.uniform(0, NX * DX, n); y = rng.uniform(0, NY * DY, n); z = np.zeros(n)
    v = rng.normal(size=(3, n)); v *= rng.uniform(0.1, 0.95, n) / np.linalg.norm(v, axis=0)
    w, q, qs = rng.uniform(0.5, 1.5, n), -1, 0.02
    F = [np.zeros((NY, NX)) for _ in range(6)]
    F[yee.EZ] = 0.3 * np.sin(2 * math.pi * np.arange(NX) / NX)[None, :] + 0 * np.zeros((NY, 1))
    g0 = yee.div_e(F, DX, DY) - D.rho(x, y, w, q, qs, NX, NY, DX, DY)
    for _ in range(steps):
        xn, yn, zn = x + v[0] * dt, y + v[1] * dt, z + v[2] * dt
        J = D.deposit(x, y, z, xn, yn, zn, w, q, qs, dt, NX, NY, DX, DY)
        yee.advance(F, DX, DY, dt, 1, J)
        x, y, z = xn, yn, zn
    g1 = yee.div_e(F, DX, DY) - D.rho(x, y, w, q, qs, NX, NY, DX, DY)
    assert np.abs(F[yee.EX]).max() > 0.01 and np.abs(F[yee.EY]).max() > 0.01   # the current drove fields
    assert np.abs(g1 - g0).max() < 1e-11 * (np.abs(g0).max() + 1)
    assert np.abs(yee.div_b(F, DX, DY)).max() < 1e-11

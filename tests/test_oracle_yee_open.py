"""Pins of the open x boundaries of the Yee oracle (first-order Mur condition, incoming
pulse injected through x_max), from the discrete scheme's closed forms:

  * at a Courant number of 1 (dy >> dx, y-uniform fields) the 1D Yee scheme transports
    exactly and the Mur factor vanishes: the injected pulse inside the grid equals the
    analytic wave, and once it has left through x_min nothing is left behind;
  * at Courant numbers 0.5 and 0.8, a quasi-monochromatic pulse leaving through either
    side reflects with the amplitude of the discrete reflection coefficient of the
    condition, R = (a + k z a - k - z)/(z - 1/a - k z/a + k), z = exp(i w dt),
    a = exp(i k~ dx) with the numerical wavenumber sin(w dt/2) = nu sin(k~ dx/2),
    k = (dt - dx)/(dt + dx) (both polarisations);
  * injection at Courant 0.5: the pulse enters at its amplitude and the grid behind it is
    left empty to the level of R;
  * a focused 2D pulse crossing the box leaves at most a small fraction of its energy
    (periodic boundaries keep all of it);
  * a beam injected on the axis of a grid symmetric in y stays mirror-symmetric (Ey, Bz
    even, Ex odd), which fixes where each component's incoming value is taken (Ey and Bz
    half a cell off the node rows).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import yee


def _plane(nx, ny, dx, dy, g, direction):
    """Ey = g(x -/+ t), Bz = +/- Ey (y-uniform wave along +x (direction=1) or -x (-1)) at
    t = 0 on the staggered positions."""
    F = [np.zeros((ny, nx)) for _ in range(6)]
    xi = np.arange(nx) * dx
    F[yee.EY][:] = g(xi)[None, :]
    F[yee.BZ][:] = direction * g(xi + 0.5 * dx)[None, :]
    return F


def _envelope(centre, ncyc):
    L = 2 * math.pi * ncyc

    def g(x):
        u = (x - centre + L / 2) / L
        return np.where((u > 0) & (u < 1), np.sin(math.pi * u) ** 2 * np.sin(x - centre), 0.0)
    return g, L


def _discrete_R(nu, dx, w=1.0):
    dt = nu * dx
    kt = 2 / dx * math.asin(math.sin(w * dt / 2) / nu)
    z, a = complex(math.cos(w * dt), math.sin(w * dt)), complex(math.cos(kt * dx), math.sin(kt * dx))
    k = (dt - dx) / (dt + dx)
    return abs((a + k * z * a - k - z) / (z - 1 / a - k * z / a + k))


def test_injection_and_exit_are_exact_at_courant_one():
    nx, ny = 300, 4
    dx = 2 * math.pi / 20
    dy = 1e3 * dx
    dt = (1 - 1e-9) / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    xmax = (nx - 1) * dx
    spec = {"kind": W.FIELD_PW, "circular": 0, "a0": 1.0, "ncycles": 3.0, "phase0": 0.0, "pol_angle": 0.0,
            "phi_start": xmax}
    F = [np.zeros((ny, nx)) for _ in range(6)]
    yee.advance(F, dx, dy, dt, 200, bc={"open_x": True, "incoming": spec, "gx0": 0.0, "gy0": 0.0, "t0": 0.0})
    t = 200 * dt
    want = np.array([oracle.field_eval(spec, t, (i * dx, 0.0, 0.0))[0][1] for i in range(nx)])
    assert np.abs(want).max() > 0.99
    assert np.abs(F[yee.EY][0] - want).max() < 2e-6
    yee.advance(F, dx, dy, dt, 500, bc={"open_x": True, "incoming": spec, "gx0": 0.0, "gy0": 0.0, "t0": t})
    assert max(np.abs(f).max() for f in F) < 1e-8


@pytest.mark.parametrize("nu", [0.5, 0.8])
@pytest.mark.parametrize("direction", [-1, 1])
def test_reflection_is_the_discrete_mur_coefficient(nu, direction):
    nx, ny = 1000, 2
    dx = 2 * math.pi / 20
    dy = 1e3 * dx
    dt = nu * dx
    g, L = _envelope(500 * dx, 30)
    F = _plane(nx, ny, dx, dy, g, direction)
    steps = int((500 * dx + L / 2 + 200 * dx) / dt)         # out through one side and back 200 cells
    yee.advance(F, dx, dy, dt, steps, bc={"open_x": True, "incoming": None, "gx0": 0.0, "gy0": 0.0, "t0": 0.0})
    R = _discrete_R(nu, dx)
    assert 1e-3 < R < 1e-2
    assert np.abs(F[yee.EY]).max() == pytest.approx(R, rel=0.03)
    # the other polarisation (Ez, By) sees the same condition
    G0 = _plane(nx, ny, dx, dy, g, direction)
    G = [np.zeros((ny, nx)) for _ in range(6)]
    G[yee.EZ] = G0[yee.EY]
    G[yee.BY] = -G0[yee.BZ]             # (Ez, By) wave along +/-x: By = -/+ Ez
    yee.advance(G, dx, dy, dt, steps, bc={"open_x": True, "incoming": None, "gx0": 0.0, "gy0": 0.0, "t0": 0.0})
    assert np.abs(G[yee.EZ]).max() == pytest.approx(R, rel=0.03)


def test_injection_at_courant_one_half_leaves_nothing_behind():
    nx, ny = 600, 2
    dx = 2 * math.pi / 20
    dy = 1e3 * dx
    dt = 0.5 * dx
    xmax = (nx - 1) * dx
    spec = {"kind": W.FIELD_PW, "circular": 0, "a0": 1.0, "ncycles": 20.0, "phase0": 0.0, "pol_angle": 0.0,
            "phi_start": xmax}
    L = 2 * math.pi * 20
    steps = int((L + 100 * dx) / dt)                        # fully inside, tail 100 cells from x_max
    F = [np.zeros((ny, nx)) for _ in range(6)]
    yee.advance(F, dx, dy, dt, steps, bc={"open_x": True, "incoming": spec, "gx0": 0.0, "gy0": 0.0, "t0": 0.0})
    ey = F[yee.EY][0]
    assert np.abs(ey).max() == pytest.approx(1.0, abs=0.02)
    behind = ey[nx - 80:]
    assert np.abs(behind).max() < 2 * _discrete_R(0.5, dx)


def test_focused_pulse_crosses_the_box():
    nx, ny = 240, 128
    dx = dy = 2 * math.pi / 16
    dt = 0.6 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    gx0, gy0 = 0.0, -0.5 * ny * dy
    xmax = gx0 + (nx - 1) * dx
    spec = {"kind": W.FIELD_GAUSS, "circular": 0, "a0": 1.0, "ncycles": 4.0, "phase0": 0.0, "pol_angle": 0.0,
            "w0": 6 * math.pi, "x_focus": gx0 + 0.5 * nx * dx, "phi_start": xmax}
    L = 2 * math.pi * 4
    F = [np.zeros((ny, nx)) for _ in range(6)]
    bc = {"open_x": True, "incoming": spec, "gx0": gx0, "gy0": gy0, "t0": 0.0}
    n1 = int((L + 0.5 * nx * dx) / dt)                      # pulse in the middle of the box
    yee.advance(F, dx, dy, dt, n1, bc=bc)
    e_mid = yee.energy(F, dx, dy)
    assert e_mid > 0
    n2 = int((0.5 * nx * dx + 40 * dx) / dt)                # and out through x_min
    yee.advance(F, dx, dy, dt, n2, bc=dict(bc, t0=n1 * dt))
    assert yee.energy(F, dx, dy) < 2e-3 * e_mid


def test_injected_beam_keeps_the_mirror_symmetry():
    nx, ny = 60, 96
    dx = dy = 2 * math.pi / 16
    dt = 0.6 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    gx0, gy0 = 0.0, -0.5 * ny * dy                           # node rows y_j = gy0 + j dy, symmetric
    xmax = gx0 + (nx - 1) * dx
    spec = {"kind": W.FIELD_GAUSS, "circular": 0, "a0": 1.0, "ncycles": 4.0, "phase0": 0.0, "pol_angle": 0.0,
            "w0": 2 * math.pi, "x_focus": xmax, "phi_start": xmax}
    F = [np.zeros((ny, nx)) for _ in range(6)]
    yee.advance(F, dx, dy, dt, int(4 * math.pi / dt), bc={"open_x": True, "incoming": spec, "gx0": gx0,
                                                          "gy0": gy0, "t0": 0.0})
    ey, bz, ex = F[yee.EY], F[yee.BZ], F[yee.EX]
    half_rows = np.arange(ny)[::-1]                          # y_{j+1/2} -> -y_{j+1/2}
    node_rows = (ny - np.arange(ny)) % ny                    # y_j -> -y_j
    scale = np.abs(ey).max()
    assert scale > 0.5 and np.abs(ex).max() > 1e-3 * scale
    assert np.abs(ey - ey[half_rows]).max() < 1e-12 * scale
    assert np.abs(bz - bz[half_rows]).max() < 1e-12 * scale
    assert np.abs(ex + ex[node_rows]).max() < 1e-12 * scale

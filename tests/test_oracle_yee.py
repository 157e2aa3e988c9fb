"""Pins of the 2D vacuum Yee solver oracle (Sec. II.B curl equations, leapfrog of
Sec. II.F), from the discrete scheme's closed forms rather than from its own code:

  * a single Fourier mode of Ez (B = 0 at t = 0) on the periodic grid evolves exactly as
    cos(n w dt) with the Yee dispersion relation sin^2(w dt/2) = dt^2 [sin^2(kx dx/2)/dx^2
    + sin^2(ky dy/2)/dy^2] (Chebyshev recurrence of the leapfrog with split B);
  * the TE and TM families do not mix;
  * the discrete divergences of E and B are invariants of the scheme (no current);
  * a mode above the Courant limit grows (the scheme is only conditionally stable).
"""
import math

import numpy as np
import pytest

from oracle import yee


def _grid(nx=48, ny=32, dx=0.15, dy=0.2):
    x = dx * np.arange(nx)
    y = dy * np.arange(ny)
    return nx, ny, dx, dy, x[None, :], y[:, None]


@pytest.mark.parametrize("mx,my", [(1, 0), (3, 2), (7, 5), (11, 13)])
def test_tm_mode_follows_the_yee_dispersion_exactly(mx, my):
    nx, ny, dx, dy, X, Y = _grid()
    kx, ky = 2 * math.pi * mx / (nx * dx), 2 * math.pi * my / (ny * dy)
    dt = 0.9 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    F = [np.zeros((ny, nx)) for _ in range(6)]
    F[yee.EZ] = np.cos(kx * X + ky * Y) + 0 * Y
    ez0 = F[yee.EZ].copy()
    S = math.sin(kx * dx / 2) ** 2 / dx ** 2 + math.sin(ky * dy / 2) ** 2 / dy ** 2
    theta = math.acos(1 - 2 * dt * dt * S)
    for n in (1, 7, 40):
        G = [f.copy() for f in F]
        yee.advance(G, dx, dy, dt, n)
        assert np.max(np.abs(G[yee.EZ] - math.cos(n * theta) * ez0)) < 1e-12 * n
        for c in (yee.EX, yee.EY, yee.BZ):
            assert np.max(np.abs(G[c])) == 0.0        # TE family untouched


def test_divergences_are_invariants():
    rng = np.random.default_rng(8)
    nx, ny, dx, dy, _, _ = _grid(40, 28)
    dt = 0.5 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    F = [rng.normal(size=(ny, nx)) for _ in range(6)]
    db0, de0 = yee.div_b(F, dx, dy), yee.div_e(F, dx, dy)
    yee.advance(F, dx, dy, dt, 60)
    assert np.max(np.abs(yee.div_b(F, dx, dy) - db0)) < 1e-11 * np.max(np.abs(db0))
    assert np.max(np.abs(yee.div_e(F, dx, dy) - de0)) < 1e-11 * np.max(np.abs(de0))


def test_plane_wave_travels_along_minus_x_at_the_numerical_phase_velocity():
    """Ey = cos(k(x + t)), Bz = -Ey (the laser convention, wave along -x): after n steps
    the wave is the initial one shifted by the numerical phase velocity w/k."""
    nx, ny, dx, dy, X, Y = _grid(64, 4)
    k = 2 * math.pi * 4 / (nx * dx)
    dt = 0.5 * dx
    w = 2 / dt * math.asin(dt / dx * math.sin(k * dx / 2))   # 1D Yee dispersion
    # the discrete travelling wave: E at integer times on nodes, B at (i+1/2) and the same time
    F = [np.zeros((ny, nx)) for _ in range(6)]
    F[yee.EY] = np.cos(k * X) + 0 * Y
    # eigenvector of the one-step map for this mode: B at the half node, integer time,
    # amplitude -cos(w dt / 2) (from the half-step update and the dispersion relation)
    F[yee.BZ] = -math.cos(w * dt / 2) * np.cos(k * (X + dx / 2)) + 0 * Y
    n = 30
    yee.advance(F, dx, dy, dt, n)
    want = np.cos(k * X + w * n * dt) + 0 * Y
    assert np.max(np.abs(F[yee.EY] - want)) < 1e-10


def test_beyond_the_courant_limit_a_mode_grows():
    nx, ny, dx, dy, X, Y = _grid(16, 16, 0.1, 0.1)
    dt = 1.05 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    F = [np.zeros((ny, nx)) for _ in range(6)]
    F[yee.EZ] = np.cos(math.pi / dx * X + math.pi / dy * Y) + 0 * Y   # the Nyquist mode
    yee.advance(F, dx, dy, dt, 60)
    assert np.max(np.abs(F[yee.EZ])) > 10

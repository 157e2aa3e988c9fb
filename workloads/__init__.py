"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests, the smoke
check and the benchmark.

This module holds no arithmetic of the method: only random initial conditions, laser
parameters and the harness-side field fill of the 2D grid workload.  The paper uses no
public dataset; these inputs stand in for its worked examples (electron beams colliding
head-on with intense laser pulses).  Units: t in 1/omega, x in 1/k (lambda = 2 pi),
p in m c.  Random numbers come from numpy's Philox bit generator seeded per workload.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi

FIELD_NONE, FIELD_CONST, FIELD_PW, FIELD_GAUSS, FIELD_GRID2D = 0, 1, 2, 3, 4
PROC_NCS, PROC_NCS_STOKES, PROC_NBW, PROC_VB = 1, 2, 4, 8


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def beam(n: int, *, seed: int, gamma0: float, gamma_rel_spread: float, divergence: float,
         x_mean: float, x_sigma: float, r_sigma: float, spin: str = "y", id0: int = 0) -> dict:
    """Electron bunch moving along +x.  gamma ~ N(gamma0, rel*gamma0), angles ~ N(0, div),
    x ~ N(x_mean, x_sigma), y, z ~ N(0, r_sigma).  spin: 'y' (+y), 'x' (+x, longitudinal)
    or 'iso' (isotropic unit vectors, an unpolarised beam)."""
    g = _rng(seed)
    gam = g.normal(gamma0, gamma_rel_spread * gamma0, n)
    gam = np.maximum(gam, 2.0)
    ty = g.normal(0.0, divergence, n)
    tz = g.normal(0.0, divergence, n)
    pm = np.sqrt(gam * gam - 1.0)
    nrm = np.sqrt(1.0 + ty * ty + tz * tz)
    st = {
        "x": g.normal(x_mean, x_sigma, n),
        "y": g.normal(0.0, r_sigma, n),
        "z": g.normal(0.0, r_sigma, n),
        "px": pm / nrm, "py": pm * ty / nrm, "pz": pm * tz / nrm,
        "w": np.ones(n),
        "id": np.arange(id0, id0 + n, dtype=np.uint64),
    }
    if spin == "iso":
        v = g.normal(size=(3, n))
        v /= np.linalg.norm(v, axis=0)
        st["sx"], st["sy"], st["sz"] = v[0], v[1], v[2]
    elif spin == "x":
        st["sx"], st["sy"], st["sz"] = np.ones(n), np.zeros(n), np.zeros(n)
    else:
        st["sx"], st["sy"], st["sz"] = np.zeros(n), np.ones(n), np.zeros(n)
    return st


def photons(n: int, *, seed: int, eps0: float, eps_rel_spread: float, divergence: float,
            x_mean: float, x_sigma: float, r_sigma: float, id0: int) -> dict:
    """Gamma photons moving along +x with random linear/circular polarisation states."""
    g = _rng(seed)
    eps = np.maximum(g.normal(eps0, eps_rel_spread * eps0, n), 3.0)
    ty = g.normal(0.0, divergence, n)
    tz = g.normal(0.0, divergence, n)
    nrm = np.sqrt(1.0 + ty * ty + tz * tz)
    kx, ky, kz = eps / nrm, eps * ty / nrm, eps * tz / nrm
    # polarisation basis vector e1: unit, perpendicular to k (Gram-Schmidt of +y)
    e = np.stack([np.zeros(n), np.ones(n), np.zeros(n)])
    kk = np.stack([kx, ky, kz]) / eps
    e = e - kk * np.sum(e * kk, axis=0)
    e /= np.linalg.norm(e, axis=0)
    xi = g.normal(size=(3, n))
    xi /= np.linalg.norm(xi, axis=0)
    xi *= g.uniform(0.0, 1.0, n)
    return {
        "x": g.normal(x_mean, x_sigma, n), "y": g.normal(0.0, r_sigma, n), "z": g.normal(0.0, r_sigma, n),
        "kx": kx, "ky": ky, "kz": kz, "w": np.ones(n),
        "xi1": xi[0], "xi2": xi[1], "xi3": xi[2],
        "e1x": e[0], "e1y": e[1], "e1z": e[2],
        "id": np.arange(id0, id0 + n, dtype=np.uint64),
        "alive": np.ones(n, np.uint8),
    }


# --------------------------------------------------------------------------- configurations
def c1(n: int = 10_000, start_step: int = 0) -> dict:
    """Plain FP64 method: 1e4 electrons, gamma0 = 1000 (5 %), 1 mrad, spins +y, head-on
    with a linearly polarised plane wave (lambda = 1 um, a0 = 20, sin^2 envelope of 8
    cycles), dt = T0/200, 3000 steps, NCS with spin flip, Philox seed 1.  start_step > 0
    places the bunch where it would be at that step (ballistic, at c)."""
    dt = TWO_PI / 200
    return {
        "name": "c1_pw_lp_a0_20_gamma1000",
        "leptons": beam(n, seed=101, gamma0=1000.0, gamma_rel_spread=0.05, divergence=1e-3,
                        x_mean=-4 * math.pi + start_step * dt, x_sigma=math.pi, r_sigma=TWO_PI, spin="y"),
        "field": {"kind": FIELD_PW, "circular": 0, "a0": 20.0, "ncycles": 8.0, "phase0": 0.0,
                  "pol_angle": 0.0, "phi_start": 0.0},
        "dt": dt, "steps": 3000, "procs": PROC_NCS, "seed": 1, "next_id": 1 << 40, "start_step": start_step,
    }


def c2(n: int = 10_000_000, start_step: int = 0) -> dict:
    """Mixed precision workload: 1e7 electrons, gamma0 = 2000 (10 %), 1 mrad, unpolarised,
    circularly polarised focused pulse (w0 = 3 um, a0 = 100, 10 cycles), dt = T0/500,
    NCS with photon Stokes output.  The bunch centre meets the pulse centre at the focus
    at t = 10 pi (step 2500)."""
    dt = TWO_PI / 500
    return {
        "name": "c2_gauss_cp_a0_100_gamma2000",
        "leptons": beam(n, seed=202, gamma0=2000.0, gamma_rel_spread=0.10, divergence=1e-3,
                        x_mean=-10 * math.pi + start_step * dt, x_sigma=TWO_PI, r_sigma=TWO_PI, spin="iso"),
        "field": {"kind": FIELD_GAUSS, "circular": 1, "a0": 100.0, "ncycles": 10.0, "phase0": 0.0,
                  "pol_angle": 0.0, "w0": 3 * TWO_PI, "x_focus": 0.0, "phi_start": 0.0},
        "dt": dt, "steps": 6000, "procs": PROC_NCS | PROC_NCS_STOKES, "seed": 2,
        "next_id": 1 << 40, "interaction_step": 2500, "start_step": start_step,
    }


def c3(n: int = 1_000_000, nx: int = 2048, ny: int = 512) -> dict:
    """Cascade workload: 1e6 electrons, gamma0 = 4000, counter-propagating linearly
    polarised a0 = 300 pulse sampled on a 2D Yee grid (2048 x 512 cells, 40 cells per
    lambda, fp32), NCS + photon Stokes + NBW + vacuum birefringence."""
    dx = TWO_PI / 40
    return {
        "name": "c3_grid2d_lp_a0_300_gamma4000",
        "leptons": beam(n, seed=303, gamma0=4000.0, gamma_rel_spread=0.05, divergence=1e-3,
                        x_mean=-6 * math.pi, x_sigma=math.pi, r_sigma=math.pi, spin="iso"),
        "grid": {"nx": nx, "ny": ny, "dx": dx, "dy": dx, "gx0": -0.5 * nx * dx, "gy0": -0.5 * ny * dx},
        "pulse": {"a0": 300.0, "ncycles": 8.0, "w0": 3 * TWO_PI, "phi_start": -16 * math.pi},
        "dt": TWO_PI / 500, "steps": 4000,
        "procs": PROC_NCS | PROC_NCS_STOKES | PROC_NBW | PROC_VB, "seed": 3, "next_id": 1 << 40,
    }


def c4(n_collisions: int = 64, n_min: float = 1e3, n_max: float = 2e6, start_step: int = 0, seed: int = 4) -> dict:
    """Batching: independent beam-laser collisions of uneven sizes, N_i = floor(10^U(log10
    n_min, log10 n_max)) (log-uniform), a0 ~ U(10, 200), gamma0 ~ U(500, 5000) with 5 %
    spread, linear or circular polarisation with probability 1/2, each a sin^2 plane-wave
    pulse of 8 cycles at its own random polarisation angle; dt = T0/400, NCS with photon
    Stokes.  The collisions are concatenated into one list (ids disjoint); `segments`
    gives (begin, end, field) per collision.  At `start_step` every bunch centre sits at
    the middle of its pulse (phase 8 pi)."""
    dt = TWO_PI / 400
    g = _rng(seed)
    sizes = np.floor(10.0 ** g.uniform(math.log10(n_min), math.log10(n_max), n_collisions)).astype(np.int64)
    a0s = g.uniform(10.0, 200.0, n_collisions)
    gammas = g.uniform(500.0, 5000.0, n_collisions)
    circ = g.uniform(0.0, 1.0, n_collisions) < 0.5
    pol = g.uniform(0.0, math.pi, n_collisions)
    t0 = start_step * dt
    parts, segs, begin = [], [], 0
    for k in range(n_collisions):
        m = int(sizes[k])
        st = beam(m, seed=1000 + seed * 100 + k, gamma0=float(gammas[k]), gamma_rel_spread=0.05, divergence=1e-3,
                  x_mean=4 * TWO_PI - t0, x_sigma=math.pi, r_sigma=TWO_PI, spin="iso", id0=begin)
        parts.append(st)
        field = {"kind": FIELD_PW, "circular": int(circ[k]), "a0": float(a0s[k]), "ncycles": 8.0, "phase0": 0.0,
                 "pol_angle": float(pol[k]), "phi_start": 0.0}
        segs.append((begin, begin + m, field))
        begin += m
    leptons = {key: np.concatenate([p[key] for p in parts]) for key in parts[0]}
    return {
        "name": f"c4_{n_collisions}_collisions_pw",
        "leptons": leptons, "segments": segs, "sizes": sizes.tolist(),
        "dt": dt, "steps": 6000, "procs": PROC_NCS | PROC_NCS_STOKES, "seed": seed, "next_id": 1 << 40,
        "start_step": start_step,
    }


def grid_fill(grid: dict, pulse: dict, t: float) -> list:
    """Harness fill of the six staggered field arrays (fp32, row-major [ny][nx]) with a
    linearly polarised (along y) pulse travelling along -x: transverse Gaussian profile
    exp(-y^2/w0^2), sin^2 envelope over the phase t + x - phi_start in [0, 2 pi ncycles],
    E_y = a0 env cos(phase), B_z = -E_y.  Staggering: Ex (i+1/2, j), Ey (i, j+1/2),
    Ez (i, j), Bx (i, j+1/2), By (i+1/2, j), Bz (i+1/2, j+1/2)."""
    nx, ny, dx, dy = grid["nx"], grid["ny"], grid["dx"], grid["dy"]
    x0, y0 = grid["gx0"], grid["gy0"]
    L = TWO_PI * pulse["ncycles"]

    def ey_at(xs, ys):
        ph = t + xs - pulse["phi_start"]
        env = np.where((ph >= 0) & (ph <= L), np.sin(np.pi * ph / L) ** 2, 0.0)
        return pulse["a0"] * env * np.cos(ph) * np.exp(-(ys ** 2) / pulse["w0"] ** 2)

    xi = x0 + dx * np.arange(nx)
    yj = y0 + dy * np.arange(ny)
    Ey = ey_at(xi[None, :], yj[:, None] + 0.5 * dy)
    Bz = -ey_at(xi[None, :] + 0.5 * dx, yj[:, None] + 0.5 * dy)
    z = np.zeros((ny, nx), np.float32)
    return [z, Ey.astype(np.float32), z.copy(), z.copy(), z.copy(), Bz.astype(np.float32)]

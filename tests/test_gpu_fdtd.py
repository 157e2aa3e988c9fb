"""GPU 2D Yee solver (qed_field_advance, Sec. II.B / II.F) against the FP64 oracle
(oracle/yee.py) on the same float32 initial fields: within FP32 rounding of the field
scale; the exact Fourier-mode evolution of the scheme; invariant divergence; the laser
of the cascade workload propagating along -x at c; open x boundaries with a plane wave or
a focused pulse injected through x_max (with and without a current), against the oracle
and leaving an empty box behind; argument checks."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import yee

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-fdtd] {msg}", flush=True)


def _ctx():
    return Q.Context(dt=0.01, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)


def _grid(F, dx, dy):
    ny, nx = F[0].shape
    return {"grid": [torch.as_tensor(np.ascontiguousarray(f, dtype=np.float32)).cuda() for f in F],
            "nx": nx, "ny": ny, "dx": dx, "dy": dy}


@pytest.mark.parametrize("nx,ny", [(97, 40), (300, 7)])
def test_yee_matches_oracle(nx, ny):
    _say(f"random fields {nx}x{ny}")
    rng = np.random.default_rng(nx)
    dx, dy = 0.16, 0.21
    dt = 0.7 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    F32 = [rng.normal(size=(ny, nx)).astype(np.float32) for _ in range(6)]
    g = _grid(F32, dx, dy)
    _ctx().field_advance(g, dt, 25)
    F = [f.astype(np.float64) for f in F32]
    yee.advance(F, dx, dy, dt, 25)
    scale = max(np.max(np.abs(f)) for f in F)
    for c in range(6):
        got = g["grid"][c].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - F[c])) < 2e-5 * scale, c


def test_tm_mode_and_divergence_on_the_gpu():
    _say("mode")
    nx, ny, dx, dy = 64, 48, 0.15, 0.2
    mx, my = 5, 3
    kx, ky = 2 * math.pi * mx / (nx * dx), 2 * math.pi * my / (ny * dy)
    dt = 0.9 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    X, Y = dx * np.arange(nx)[None, :], dy * np.arange(ny)[:, None]
    F = [np.zeros((ny, nx)) for _ in range(6)]
    F[yee.EZ] = np.cos(kx * X + ky * Y)
    g = _grid(F, dx, dy)
    n = 60
    _ctx().field_advance(g, dt, n)
    S = math.sin(kx * dx / 2) ** 2 / dx ** 2 + math.sin(ky * dy / 2) ** 2 / dy ** 2
    theta = math.acos(1 - 2 * dt * dt * S)
    ez = g["grid"][yee.EZ].cpu().numpy()
    assert np.max(np.abs(ez - math.cos(n * theta) * F[yee.EZ])) < 2e-5
    G = [t.cpu().numpy().astype(np.float64) for t in g["grid"]]
    assert np.max(np.abs(yee.div_b(G, dx, dy))) < 1e-4   # zero initially; FP32 rounding only


def test_cascade_laser_propagates_along_minus_x():
    """The cascade workload's pulse, filled at t = 0 and advanced 200 steps on the
    2048 x 512 grid, against the harness fill at t = 200 dt: the same pulse moved by 200 dt
    along -x, up to the grid's numerical dispersion (40 cells per wavelength)."""
    _say("cascade laser")
    cfg = W.c3(n=10)
    grid, pulse = cfg["grid"], dict(cfg["pulse"])
    pulse["phi_start"] = -pulse["ncycles"] * math.pi
    g = dict(grid, grid=[torch.as_tensor(c).cuda() for c in W.grid_fill(grid, pulse, 0.0)])
    n = 200
    _ctx().field_advance(g, cfg["dt"], n)
    want = W.grid_fill(grid, pulse, n * cfg["dt"])
    a0 = pulse["a0"]
    for c in (1, 5):   # Ey, Bz
        got = g["grid"][c].cpu().numpy()
        assert np.max(np.abs(got - want[c])) < 0.03 * a0, c
        assert np.max(np.abs(got)) > 0.5 * a0


def test_field_advance_arguments_are_checked():
    F = [np.zeros((8, 8)) for _ in range(6)]
    g = _grid(F, 0.1, 0.1)
    ctx = _ctx()
    with pytest.raises(Q.QedError):
        ctx.field_advance(g, 0.08, 1)                # beyond the Courant limit (0.0707)
    with pytest.raises(Q.QedError):
        ctx.field_advance(dict(g, nx=1), 0.01, 1)


def _open_case(nx, ny, dx, dy, spec_kind):
    gx0, gy0 = 0.0, -0.5 * ny * dy
    xmax = gx0 + (nx - 1) * dx
    spec = {"kind": spec_kind, "circular": 0, "a0": 2.0, "ncycles": 3.0, "phase0": 0.3, "pol_angle": 0.4,
            "w0": 2 * math.pi, "x_focus": gx0 + 0.5 * nx * dx, "phi_start": xmax + 0.7}
    return gx0, gy0, spec


@pytest.mark.parametrize("kind,with_current", [(W.FIELD_GAUSS, False), (W.FIELD_PW, True)])
def test_open_boundaries_match_oracle(kind, with_current):
    _say(f"open boundaries kind {kind} current {with_current}")
    nx, ny, dx, dy = 90, 48, 2 * math.pi / 16, 2 * math.pi / 14
    dt = 0.6 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    gx0, gy0, spec = _open_case(nx, ny, dx, dy, kind)
    rng = np.random.default_rng(7)
    F32 = [(0.01 * rng.normal(size=(ny, nx))).astype(np.float32) for _ in range(6)]
    J32 = [(0.05 * rng.normal(size=(ny, nx))).astype(np.float32) for _ in range(3)] if with_current else None
    g = _grid(F32, dx, dy)
    bc = {"open_x": 1, "incoming": spec, "gx0": gx0, "gy0": gy0, "t0": 1.5}
    steps = 160
    cur = [torch.as_tensor(j).cuda() for j in J32] if with_current else None
    _ctx().field_advance(g, dt, steps, current=cur, bc=bc)
    F = [f.astype(np.float64) for f in F32]
    yee.advance(F, dx, dy, dt, steps, [j.astype(np.float64) for j in J32] if with_current else None,
                bc={"open_x": True, "incoming": spec, "gx0": gx0, "gy0": gy0, "t0": 1.5})
    scale = max(np.max(np.abs(f)) for f in F)
    assert scale > 0.5                                    # the pulse came in
    for c in range(6):
        got = g["grid"][c].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - F[c])) < 1e-4 * scale, c


def test_injected_pulse_leaves_an_empty_box():
    _say("pulse through the box")
    nx, ny, dx, dy = 200, 64, 2 * math.pi / 16, 2 * math.pi / 16
    dt = 0.6 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    gx0, gy0, spec = _open_case(nx, ny, dx, dy, W.FIELD_PW)
    F = [np.zeros((ny, nx), dtype=np.float32) for _ in range(6)]
    g = _grid(F, dx, dy)
    ctx = _ctx()
    L = 2 * math.pi * 3
    n1 = int((L + 0.5 * nx * dx) / dt)
    bc = {"open_x": 1, "incoming": spec, "gx0": gx0, "gy0": gy0, "t0": 0.0}
    ctx.field_advance(g, dt, n1, bc=bc)
    e_mid = sum(float((c.double() ** 2).sum()) for c in g["grid"])
    n2 = int((0.5 * nx * dx + 30 * dx) / dt)
    ctx.field_advance(g, dt, n2, bc=dict(bc, t0=n1 * dt))
    e_end = sum(float((c.double() ** 2).sum()) for c in g["grid"])
    # what is left is the reflection of the condition: |R|^2 of the energy at the carrier
    # (discrete reflection coefficient of the first-order Mur condition), more for the
    # shorter wavelengths of a three-cycle pulse
    nu = dt / dx
    kt = 2 / dx * math.asin(math.sin(dt / 2) / nu)
    z, a = complex(math.cos(dt), math.sin(dt)), complex(math.cos(kt * dx), math.sin(kt * dx))
    k = (dt - dx) / (dt + dx)
    R = abs((a + k * z * a - k - z) / (z - 1 / a - k * z / a + k))
    assert e_mid > 100 and e_end < 3 * R * R * e_mid


def test_open_boundary_arguments_are_checked():
    F = [np.zeros((8, 8)) for _ in range(6)]
    ctx = _ctx()
    bc = {"open_x": 1, "incoming": None, "gx0": 0.0, "gy0": 0.0, "t0": 0.0}
    with pytest.raises(Q.QedError):
        ctx.field_advance(_grid(F, 0.1, 0.1), 0.05, 1, bc=dict(bc, open_x=2))
    with pytest.raises(Q.QedError):
        ctx.field_advance(_grid([np.zeros((8, 3)) for _ in range(6)], 0.1, 0.1), 0.05, 1, bc=bc)
    with pytest.raises(Q.QedError):
        ctx.field_advance(_grid(F, 0.1, 0.1), 0.05, 1, bc=dict(bc, incoming={"kind": W.FIELD_CONST}))
    with pytest.raises(Q.QedError):
        ctx.field_advance(_grid(F, 0.1, 0.1), 0.05, 1, bc=dict(bc, t0=float("inf")))

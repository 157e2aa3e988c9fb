"""GPU 2D vacuum Yee solver (qed_field_advance, Sec. II.B / II.F) against the FP64 oracle
(oracle/yee.py) on the same float32 initial fields: within FP32 rounding of the field
scale; the exact Fourier-mode evolution of the scheme; invariant divergence; the laser
of the cascade workload propagating along -x at c; argument checks."""
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

"""GPU charge-conserving current deposition (qed_deposit_current, Sec. II.C) against the
FP64 oracle (oracle/deposit.py), and the field solver with the current term:

  * parity on the same positions and weights, node by node within FP32 rounding of the
    contributions (periodic wrap, positions outside the box, both charges, a grid origin,
    particles appended after the start of the step left out);
  * at the size of the cascade workload (1e6 electrons, 2048 x 512 grid): total current
    = sum Q v and the discrete continuity equation against the oracle's charge density;
    the binned path gives the same bits on a second run;
  * the solver's E update with J against the oracle's;
  * a self-consistent loop on the GPU (gather from the grid, push, deposit, advance):
    div E - rho keeps its initial value (Gauss's law);
  * moves of a cell or more are skipped and flagged; argument checks.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import deposit as D
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
    print(f"[gpu-deposit] {msg}", flush=True)


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _leptons(x, y, z, w, charge, capacity=None):
    n = len(x)
    st = {k: np.zeros(n) for k in ("px", "py", "pz", "sx", "sy", "sz")}
    st.update(x=x, y=y, z=z, w=w, id=np.arange(n, dtype=np.uint64))
    return Q.Leptons.from_state(st, capacity=capacity or n, charge=charge, precision=Q.QED_MIXED)


def _zeros(ny, nx):
    return [torch.zeros((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]


def _random_moves(n, nx, ny, dx, dy, gx0, gy0, seed, frac=0.97):
    rng = np.random.default_rng(seed)
    xa = gx0 + rng.uniform(-3 * dx, (nx + 3) * dx, n)
    ya = gy0 + rng.uniform(-3 * dy, (ny + 3) * dy, n)
    za = rng.normal(0, 1, n)
    xb = xa + rng.uniform(-frac, frac, n) * dx
    yb = ya + rng.uniform(-frac, frac, n) * dy
    zb = za + rng.uniform(-0.05, 0.05, n)
    w = rng.uniform(0.2, 1.0, n)
    return xa, ya, za, xb, yb, zb, w


@pytest.mark.parametrize("charge,gx0,gy0,nx,ny", [(-1, 0.0, 0.0, 64, 48), (1, -5.1, 2.3, 37, 20),
                                                  (-1, 0.4, -0.2, 5, 3),          # smaller than a tile's window
                                                  (1, 0.0, 0.0, 2048, 1100)])     # 32 x 32-node tiles
def test_deposit_matches_oracle(charge, gx0, gy0, nx, ny):
    _say(f"parity charge {charge} grid {nx}x{ny}")
    dx, dy, dt, qs = 0.19, 0.23, 0.05, 0.7
    n, n0 = 3000, 2600                               # the last 400 were appended during the step
    xa, ya, za, xb, yb, zb, w = _random_moves(n, nx, ny, dx, dy, gx0, gy0, seed=nx)
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = _leptons(xb, yb, zb, w, charge, capacity=n + 100)
    start = (_dev(xa), _dev(ya), _dev(za), torch.tensor([n0], dtype=torch.int64, device="cuda"))
    J = _zeros(ny, nx)
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": gx0, "gy0": gy0}
    ctx.deposit_current([(L, start)], grid, J, qs)
    assert ctx.read_status() == 0
    want = D.deposit(xa[:n0], ya[:n0], za[:n0], xb[:n0], yb[:n0], zb[:n0], w[:n0], charge, qs, dt, nx, ny, dx, dy,
                     gx0, gy0)
    # binned path: exact fixed-point sums (quantum 2^-32 of the largest contribution) and
    # one FP32 rounding of each node's value
    qmax = qs * w.max()
    scale = (qmax / (dy * dt), qmax / (dx * dt), qmax * 0.05 / dt / (dx * dy))
    for c in range(3):
        got = J[c].cpu().numpy().astype(np.float64)
        assert np.abs(want[c]).max() > 0.3 * scale[c]
        assert np.all(np.abs(got - want[c]) < 1e-6 * scale[c] + 1.2e-7 * np.abs(want[c])), c
    # deposit adds: a second call doubles
    ctx.deposit_current([(L, start)], grid, J, qs)
    got2 = J[0].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got2 - 2 * want[0]) < 2e-6 * scale[0] + 3e-7 * np.abs(want[0]))


def test_two_species_in_one_call():
    """Electrons and positrons (separate lists, each with its own start count) in one call:
    the oracle's deposit of the two added."""
    _say("two species")
    nx, ny, dx, dy, dt, qs = 48, 40, 0.2, 0.25, 0.05, 0.4
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    srcs, want = [], [np.zeros((ny, nx)) for _ in range(3)]
    for charge, seed, n, n0 in ((-1, 21, 2500, 2400), (1, 22, 900, 900)):
        xa, ya, za, xb, yb, zb, w = _random_moves(n, nx, ny, dx, dy, 0.0, 0.0, seed=seed)
        L = _leptons(xb, yb, zb, w, charge)
        start = (_dev(xa), _dev(ya), _dev(za), torch.tensor([n0], dtype=torch.int64, device="cuda"))
        srcs.append((L, start))
        d = D.deposit(xa[:n0], ya[:n0], za[:n0], xb[:n0], yb[:n0], zb[:n0], w[:n0], charge, qs, dt, nx, ny, dx, dy)
        for c in range(3):
            want[c] += d[c]
    J = _zeros(ny, nx)
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": 0.0, "gy0": 0.0}
    ctx.deposit_current(srcs, grid, J, qs)
    assert ctx.read_status() == 0
    scale = (qs / (dy * dt), qs / (dx * dt), qs * 0.05 / dt / (dx * dy))
    for c in range(3):
        got = J[c].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - want[c]) < 1e-6 * scale[c] + 1.2e-7 * np.abs(want[c])), c
    with pytest.raises(Q.QedError):
        ctx.deposit_current([], grid, J, qs)
    with pytest.raises(Q.QedError):
        ctx.deposit_current(srcs * 3, grid, J, qs)       # more than four sources


def test_dense_cluster_spans_several_chunks():
    """30 000 particles within three cells: tiles with more particles than one block of the
    tiled path takes, so several blocks flush into the same nodes."""
    _say("dense cluster")
    nx, ny, dx, dy, dt, qs = 80, 64, 0.2, 0.2, 0.05, 0.01
    rng = np.random.default_rng(4)
    n = 30000
    xa = 31.5 * dx + rng.uniform(-1.5, 1.5, n) * dx
    ya = 15.6 * dy + rng.uniform(-1.5, 1.5, n) * dy
    xb, yb = xa + rng.uniform(-0.9, 0.9, n) * dx, ya + rng.uniform(-0.9, 0.9, n) * dy
    za, zb = np.zeros(n), rng.uniform(-0.04, 0.04, n)
    w = rng.uniform(0.5, 1.0, n)
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = _leptons(xb, yb, zb, w, -1)
    start = (_dev(xa), _dev(ya), _dev(za), torch.tensor([n], dtype=torch.int64, device="cuda"))
    J = _zeros(ny, nx)
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": 0.0, "gy0": 0.0}
    ctx.deposit_current([(L, start)], grid, J, qs)
    want = D.deposit(xa, ya, za, xb, yb, zb, w, -1, qs, dt, nx, ny, dx, dy)
    for c in range(3):
        got = J[c].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - want[c])) < 1e-4 * np.abs(want[c]).max(), c


def test_direct_path_on_a_grid_too_large_to_tile():
    """4160 x 4160 nodes: more tiles than the tiled path handles, so one thread per particle
    adds straight to the arrays."""
    _say("direct path")
    nx = ny = 4160
    dx, dy, dt, qs = 0.1, 0.1, 0.04, 0.5
    xa, ya, za, xb, yb, zb, w = _random_moves(4000, nx, ny, dx, dy, 0.0, 0.0, seed=8)
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = _leptons(xb, yb, zb, w, 1)
    start = (_dev(xa), _dev(ya), _dev(za), torch.tensor([4000], dtype=torch.int64, device="cuda"))
    J = _zeros(ny, nx)
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": 0.0, "gy0": 0.0}
    ctx.deposit_current([(L, start)], grid, J, qs)
    assert ctx.read_status() == 0
    want = D.deposit(xa, ya, za, xb, yb, zb, w, 1, qs, dt, nx, ny, dx, dy)
    qmax = qs * w.max()
    scale = (qmax / (dy * dt), qmax / (dx * dt), qmax * 0.05 / dt / (dx * dy))
    for c in range(3):
        got = J[c].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - want[c])) < 1e-5 * scale[c], c
    del J


def test_cascade_size_moments_and_continuity():
    """1e6 electrons of the cascade workload pushed one step in its pulse on the 2048 x 512
    grid (dense beam: many particles per node), deposited; properties that hold at any size."""
    cfg = W.c3()
    grid, pulse = cfg["grid"], dict(cfg["pulse"])
    pulse["phi_start"] = -pulse["ncycles"] * math.pi
    comps = [torch.as_tensor(c).cuda() for c in W.grid_fill(grid, pulse, 0.0)]
    spec = dict(kind=Q.FIELD_GRID2D, grid=comps, **grid)
    st = dict(cfg["leptons"])
    st["x"] = st["x"] - st["x"].mean()
    n = len(st["x"])
    _say(f"cascade size n={n}")
    ctx = Q.Context(dt=cfg["dt"], procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = Q.Leptons.from_state(st, charge=-1, precision=Q.QED_MIXED)
    start = ctx.save_start(L)
    ctx.push_spin(Q.whole(spec), L, 100)
    J = _zeros(grid["ny"], grid["nx"])
    qs = 1e-4
    ctx.deposit_current([(L, start)], grid, J, qs)
    assert ctx.read_status() == 0
    J2 = _zeros(grid["ny"], grid["nx"])
    ctx.deposit_current([(L, start)], grid, J2, qs)
    for c in range(3):                              # integer sums in the binned path: same bits every run
        assert torch.equal(J[c], J2[c]), c
    xa, ya, za = (t.cpu().numpy() for t in start[:3])
    xb, yb, zb, w = (getattr(L, k).cpu().numpy() for k in ("x", "y", "z", "w"))
    dt, dx, dy = cfg["dt"], grid["dx"], grid["dy"]
    Jn = [j.cpu().numpy().astype(np.float64) for j in J]
    Qw = -qs * w
    for c, d in ((0, xb - xa), (1, yb - ya), (2, zb - za)):
        want = (Qw * d).sum() / dt
        assert Jn[c].sum() * dx * dy == pytest.approx(want, rel=2e-4, abs=1e-6 * np.abs(Qw * d).sum() / dt), c
    nx, ny, g0x, g0y = grid["nx"], grid["ny"], grid["gx0"], grid["gy0"]
    r0 = D.rho(xa, ya, w, -1, qs, nx, ny, dx, dy, g0x, g0y)
    r1 = D.rho(xb, yb, w, -1, qs, nx, ny, dx, dy, g0x, g0y)
    res = (r1 - r0) / dt + D.divergence(Jn[0], Jn[1], dx, dy)
    drho = np.abs(r1 - r0).max() / dt
    assert drho > 0
    assert np.abs(res).max() < 2e-4 * drho * 40     # FP32 sums over ~1e3 contributions per node


def _both_paths(srcs, grid, qs, dt, first=None):
    """J from the binned and from the local path (fresh contexts), and the status words;
    `first`: sources of an earlier call on the same context (its J is discarded)."""
    out = []
    for path in (Q.DEPOSIT_BINNED, Q.DEPOSIT_LOCAL):
        ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
        ctx.set_deposit_path(path)
        if first is not None:
            ctx.deposit_current(first, grid, _zeros(grid["ny"], grid["nx"]), qs)
        J = _zeros(grid["ny"], grid["nx"])
        ctx.deposit_current(srcs, grid, J, qs)
        ctx.deposit_current(srcs, grid, J, qs)         # a second call adds the same again
        out.append((J, ctx.read_status()))
    return out


@pytest.mark.parametrize("order", ["sorted", "random"])
def test_local_path_equals_binned_at_cascade_size(order):
    """The cascade's 1e6 electrons pushed one step on the 2048 x 512 grid: sorted by 4 x 4-cell
    bin (blocks of 256 consecutive electrons fit their LDS windows) or in random order (every
    block too spread out: contributions straight to the 64-bit grid).  Either way the local
    path adds the binned path's integer sums, so J is the same bit for bit."""
    cfg = W.c3()
    grid, pulse = cfg["grid"], dict(cfg["pulse"])
    pulse["phi_start"] = -pulse["ncycles"] * math.pi
    comps = [torch.as_tensor(c).cuda() for c in W.grid_fill(grid, pulse, 0.0)]
    spec = dict(kind=Q.FIELD_GRID2D, grid=comps, **grid)
    st = dict(cfg["leptons"])
    st["x"] = st["x"] - st["x"].mean()
    n = len(st["x"])
    _say(f"local vs binned, {order}, n={n}")
    if order == "random":
        perm = np.random.default_rng(3).permutation(n)
        st = {k: v[perm] for k, v in st.items()}
    ctx = Q.Context(dt=cfg["dt"], procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = Q.Leptons.from_state(st, charge=-1, precision=Q.QED_MIXED)
    if order == "sorted":
        Ls = Q.Leptons(n, -1, precision=Q.QED_MIXED)
        ctx.sort_leptons(L, Ls, spec)
        L = Ls
    start = ctx.save_start(L)
    ctx.push_spin(Q.whole(spec), L, 100)
    (Jb, sb), (Jl, sl) = _both_paths([(L, start)], grid, 1e-4, cfg["dt"])
    assert sb == sl == 0
    for c in range(3):
        assert float(Jb[c].abs().max()) > 0
        assert torch.equal(Jb[c], Jl[c]), c


@pytest.mark.parametrize("nx,ny,gx0,gy0", [(37, 20, -5.1, 2.3), (5, 3, 0.4, -0.2), (256, 64, 0.0, 0.0)])
def test_local_path_equals_binned_small(nx, ny, gx0, gy0):
    """Two sources of different charge, particles across the periodic seams and outside the
    box, a few moves of more than a cell (skipped and flagged by both), appended particles
    left out; clusters sorted by cell beside scattered ones: the same J bit for bit."""
    _say(f"local vs binned {nx}x{ny}")
    dx, dy, dt, qs = 0.19, 0.23, 0.05, 0.7
    srcs = []
    for charge, seed, n, n0 in ((-1, 31, 5000, 4600), (1, 32, 3000, 3000)):
        xa, ya, za, xb, yb, zb, w = _random_moves(n, nx, ny, dx, dy, gx0, gy0, seed=seed)
        k = n // 2                                         # first half: a cluster, sorted by cell
        rng = np.random.default_rng(seed + 100)
        xa[:k] = gx0 + (nx * 0.5 + rng.normal(0, 2.0, k)) * dx
        ya[:k] = gy0 + (ny * 0.5 + rng.normal(0, 2.0, k)) * dy
        o = np.lexsort((np.floor((xa[:k] - gx0) / dx), np.floor((ya[:k] - gy0) / dy)))
        xa[:k], ya[:k] = xa[:k][o], ya[:k][o]
        xb[:k] = xa[:k] + rng.uniform(-0.9, 0.9, k) * dx
        yb[:k] = ya[:k] + rng.uniform(-0.9, 0.9, k) * dy
        xb[k + 7] = xa[k + 7] + 1.5 * dx                    # skipped: a move of more than a cell
        L = _leptons(xb, yb, zb, w, charge)
        srcs.append((L, (_dev(xa), _dev(ya), _dev(za), torch.tensor([n0], dtype=torch.int64, device="cuda"))))
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": gx0, "gy0": gy0}
    (Jb, sb), (Jl, sl) = _both_paths(srcs, grid, qs, dt)
    assert sb == sl == Q.ST_DEPOSIT
    for c in range(3):
        assert torch.equal(Jb[c], Jl[c]), c
    # after a call with 8x the weights (a coarser fixed-point scale) each call sets its own
    # scale: the same bits as the binned path again
    heavy = []
    for L, start in srcs:
        H = Q.Leptons(L.capacity, L.charge, precision=Q.QED_MIXED)
        for k in ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz", "id"):
            getattr(H, k).copy_(getattr(L, k))
        H.w.mul_(8.0)
        H.count_t.copy_(L.count_t)
        heavy.append((H, start))
    (Jb2, _), (Jl2, _) = _both_paths(srcs, grid, qs, dt, first=heavy)
    for c in range(3):
        assert torch.equal(Jb2[c], Jl2[c]) and torch.equal(Jb2[c], Jb[c]), c
    with pytest.raises(Q.QedError):
        Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED).set_deposit_path(2)


def test_solver_current_term_matches_oracle():
    _say("solver with J")
    rng = np.random.default_rng(3)
    nx, ny, dx, dy = 70, 33, 0.16, 0.21
    dt = 0.7 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    F32 = [rng.normal(size=(ny, nx)).astype(np.float32) for _ in range(6)]
    J32 = [rng.normal(size=(ny, nx)).astype(np.float32) for _ in range(3)]
    g = {"grid": [_dev(f, torch.float32) for f in F32], "nx": nx, "ny": ny, "dx": dx, "dy": dy}
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    ctx.field_advance(g, dt, 10, current=[_dev(j, torch.float32) for j in J32])
    F = [f.astype(np.float64) for f in F32]
    yee.advance(F, dx, dy, dt, 10, [j.astype(np.float64) for j in J32])
    scale = max(np.max(np.abs(f)) for f in F)
    for c in range(6):
        assert np.max(np.abs(g["grid"][c].cpu().numpy() - F[c])) < 2e-5 * scale, c


def test_self_consistent_loop_keeps_gauss_law():
    """Gather from the grid, Boris push, deposit, advance, on the GPU for 60 steps: the
    discrete div E - rho stays at its initial value, while rho changes by far more."""
    _say("self-consistent loop")
    rng = np.random.default_rng(11)
    nx, ny = 96, 64
    dx = dy = 2 * math.pi / 20
    dt = 0.6 / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    gx0, gy0 = -0.5 * nx * dx, -0.5 * ny * dy
    n = 20000
    x = rng.normal(0, 6 * dx, n)
    y = rng.normal(0, 6 * dy, n)
    p = rng.normal(size=(3, n)) * 2.0
    w = np.full(n, 1.0)
    st = {"x": x, "y": y, "z": np.zeros(n), "px": p[0], "py": p[1], "pz": p[2], "sx": np.zeros(n),
          "sy": np.zeros(n), "sz": np.ones(n), "w": w, "id": np.arange(n, dtype=np.uint64)}
    ctx = Q.Context(dt=dt, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = Q.Leptons.from_state(st, charge=-1, precision=Q.QED_MIXED)
    comps = [torch.zeros((ny, nx), dtype=torch.float32, device="cuda") for _ in range(6)]
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": gx0, "gy0": gy0}
    spec = dict(kind=Q.FIELD_GRID2D, grid=comps, **grid)
    segs = Q.whole(spec)
    J = _zeros(ny, nx)
    qs = 2e-4
    start = ctx.save_start(L)
    x0 = L.x.cpu().numpy(); y0 = L.y.cpu().numpy()
    g0 = -D.rho(x0, y0, w, -1, qs, nx, ny, dx, dy, gx0, gy0)          # div E = 0 at the start
    for s in range(60):
        ctx.save_start(L, start)
        ctx.push_spin(segs, L, s)
        for j in J:
            j.zero_()
        ctx.deposit_current([(L, start)], grid, J, qs)
        ctx.field_advance(spec, dt, 1, current=J)
    assert ctx.read_status() == 0
    F = [c.cpu().numpy().astype(np.float64) for c in comps]
    x1 = L.x.cpu().numpy(); y1 = L.y.cpu().numpy()
    r1 = D.rho(x1, y1, w, -1, qs, nx, ny, dx, dy, gx0, gy0)
    g1 = yee.div_e(F, dx, dy) - r1
    drho = np.abs(r1 + g0).max()                    # |rho1 - rho0|
    emax = max(np.abs(F[c]).max() for c in range(3))
    _say(f"drho {drho:.3e} residual {np.abs(g1 - g0).max():.3e} Emax {emax:.3e}")
    assert drho > 0.1 * np.abs(g0).max()            # the beam spread noticeably
    assert emax > 1e-4                               # the current built up fields
    assert np.abs(g1 - g0).max() < 1e-3 * drho
    assert np.abs(yee.div_b(F, dx, dy)).max() < 1e-3 * emax / dx


def test_large_moves_are_skipped_and_flagged():
    _say("flags")
    nx = ny = 16
    dx = dy = 0.2
    ctx = Q.Context(dt=0.05, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    L = _leptons(np.array([0.5, 1.0 + dx * 1.2]), np.array([0.5, 1.0]), np.zeros(2), np.ones(2), -1)
    start = (_dev([0.5 + 0.1 * dx, 1.0]), _dev([0.5, 1.0]), _dev([0.0, 0.0]),
             torch.tensor([2], dtype=torch.int64, device="cuda"))
    J = _zeros(ny, nx)
    grid = {"nx": nx, "ny": ny, "dx": dx, "dy": dy, "gx0": 0.0, "gy0": 0.0}
    ctx.deposit_current([(L, start)], grid, J, 1.0)
    assert ctx.read_status() & Q.ST_DEPOSIT
    want = D.deposit([0.5 + 0.1 * dx], [0.5], [0.0], [0.5], [0.5], [0.0], [1.0], -1, 1.0, 0.05, nx, ny, dx, dy)
    assert np.allclose(J[0].cpu().numpy(), want[0], rtol=1e-6, atol=1e-6 * np.abs(want[0]).max())
    ctx.clear_status()
    with pytest.raises(Q.QedError):
        ctx.deposit_current([(L, start)], dict(grid, nx=1), J, 1.0)
    with pytest.raises(Q.QedError):
        ctx.deposit_current([(L, start)], dict(grid, dx=0.0), J, 1.0)
    with pytest.raises(Q.QedError):
        ctx.deposit_current([(L, start)], grid, J, float("nan"))

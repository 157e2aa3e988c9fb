"""GPU lepton step (push, T-BMT, NCS with photon Stokes) on a 2D grid against the oracle,
with the leptons in wavefront-sized clusters: the decide kernel's LDS box path, and its
global-gather fallback for wavefronts with an outlier or near the grid's edge.  FP64 to
the parity bar, mixed within single-precision error of the FP64 path; a segment that
covers part of the list (lanes outside it take no part in the box and see no field)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402

from test_gpu_parity import _close_lep, _close_pho, _ctx, _sim  # noqa: E402
from test_gpu_photon_grid import WAVE, _wave_box  # noqa: E402

DX, DY, GX0, GY0 = 0.7, 0.45, -1.3, 2.1
N = 3000
STEPS = (40, 41, 42, 43, 44)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-lepton-grid] {msg}", flush=True)


def _case(nx, ny, seed):
    """Random field values on the grid; electrons at gamma 1000 whose wavefronts sit within
    +-2.5 nodes of a centre anywhere over the grid and its border, every third wavefront
    with one outlier anywhere."""
    rng = np.random.default_rng(seed)
    comps = [rng.uniform(-300.0, 300.0, (ny, nx)).astype(np.float32) for _ in range(6)]
    st = W.beam(N, seed=seed + 1, gamma0=1000.0, gamma_rel_spread=0.05, divergence=1e-2, x_mean=0.0, x_sigma=1.0,
                r_sigma=1.0, spin="iso")
    nw = (N + WAVE - 1) // WAVE
    cx, cy = rng.uniform(-1.0, nx + 1.0, nw), rng.uniform(-1.0, ny + 1.0, nw)
    w = np.arange(N) // WAVE
    st["x"] = GX0 + DX * (cx[w] + rng.uniform(-2.5, 2.5, N))
    st["y"] = GY0 + DY * (cy[w] + rng.uniform(-2.5, 2.5, N))
    for b in range(0, nw, 3):
        lane = b * WAVE + int(rng.integers(0, min(WAVE, N - b * WAVE)))
        st["x"][lane] = GX0 + DX * rng.uniform(-3.0, nx + 2.0)
    grid = dict(nx=nx, ny=ny, dx=DX, dy=DY, gx0=GX0, gy0=GY0)
    spec_o = dict(kind=W.FIELD_GRID2D, grid=comps, **grid)
    spec_g = dict(spec_o, grid=[torch.as_tensor(c).cuda() for c in comps])
    fits = _wave_box(st["x"], st["y"], np.ones(N, np.uint8), nx, ny, DX, DY, GX0, GY0)
    one = _wave_box(st["x"], st["y"], np.ones(N, np.uint8), nx, ny, DX, DY, GX0, GY0, limit=64).sum()
    _say(f"{nx}x{ny}: {int(fits.sum())} of {len(fits)} wavefronts on the box path ({one} filled by one load)")
    assert 0.15 * len(fits) < fits.sum() < 0.9 * len(fits)
    assert one >= 3 and fits.sum() - one >= 3
    return st, spec_o, spec_g


CFG = {"dt": W.TWO_PI / 500, "procs": oracle.PROC_NCS | oracle.PROC_NCS_STOKES, "seed": 17, "next_id": 1 << 41}


def _gpu_run(st, segs, precision):
    ctx = _ctx(CFG, precision=precision)
    em = Q.Leptons.from_state(st, capacity=N, charge=-1, precision=precision)
    ep = Q.Leptons(N, 1, precision=precision)
    G = Q.Photons(20 * N, precision=precision)
    for s in STEPS:
        ctx.step(segs, em, ep, G, s)
    return ctx, em.to_numpy(), G.to_numpy()


@pytest.mark.parametrize("nx,ny", [(40, 24), (200, 30)])
def test_lepton_step_on_grid_clusters(nx, ny):
    _say(f"leptons in clusters on a {nx}x{ny} grid")
    st, spec_o, spec_g = _case(nx, ny, 300 + nx)
    f = oracle.make_field(spec_o)
    em = oracle.LeptonArrays.from_state(st, capacity=N, charge=-1)
    ep = oracle.LeptonArrays.empty(N, 1)
    G = oracle.PhotonArrays.empty(20 * N)
    sim = _sim(CFG)
    for s in STEPS:
        sim.step(f, em, ep, G, s)
    ctx, emg, Gg = _gpu_run(st, Q.whole(spec_g), Q.QED_FP64)
    _say(f"{G.count} photons")
    assert G.count > 100, G.count
    _close_lep(emg, em.view(), what="electrons")
    _close_pho(Gg, G.view(), what="photons")
    assert ctx.next_id() == sim.next_id and ctx.read_status() == 0
    # mixed: within single precision of the FP64 path (same draws; an emission decision may
    # differ only where the probability sits within rounding of the draw)
    _, emm, Gm = _gpu_run(st, Q.whole(spec_g), Q.QED_MIXED)
    assert abs(len(Gm["x"]) - len(Gg["x"])) <= 3
    pm = np.sqrt(emg["px"] ** 2 + emg["py"] ** 2 + emg["pz"] ** 2)
    dp = np.sqrt((emm["px"] - emg["px"]) ** 2 + (emm["py"] - emg["py"]) ** 2 + (emm["pz"] - emg["pz"]) ** 2) / pm
    assert np.sort(dp)[-7] < 2e-5, np.sort(dp)[-7:]     # all but at most six leptons


def test_partial_segment_on_grid():
    """A segment over [400, N - 300): leptons inside step as with the whole-list segment
    (the box of a wavefront then spans only its lanes inside), leptons outside see no field:
    momentum and spin unchanged, position advanced ballistically, no photon."""
    _say("partial segment")
    nx, ny = 200, 30
    st, _, spec_g = _case(nx, ny, 700)
    b, e = 400, N - 300
    ctx, whole, Gw = _gpu_run(st, Q.whole(spec_g), Q.QED_FP64)
    ctx2, part, Gp = _gpu_run(st, Q.segments([(b, e, spec_g)]), Q.QED_FP64)
    inside = np.zeros(N, bool)
    inside[b:e] = True
    pmag = np.sqrt(whole["px"] ** 2 + whole["py"] ** 2 + whole["pz"] ** 2)
    for k in ("px", "py", "pz"):
        assert np.max(np.abs(part[k][inside] - whole[k][inside]) / pmag[inside]) < 1e-12, k
    for k in ("sx", "sy", "sz"):
        assert np.max(np.abs(part[k][inside] - whole[k][inside])) < 1e-12, k
    for k in ("px", "py", "pz", "sx", "sy", "sz"):
        assert np.array_equal(part[k][~inside], st[k][~inside]), k
    g = np.sqrt(1.0 + st["px"] ** 2 + st["py"] ** 2 + st["pz"] ** 2)
    for k, pk in (("x", "px"), ("y", "py"), ("z", "pz")):
        want = st[k][~inside] + len(STEPS) * CFG["dt"] * st[pk][~inside] / g[~inside]
        assert np.max(np.abs(part[k][~inside] - want)) < 1e-12 * (1 + np.max(np.abs(want))), k
    # photons only from the leptons inside: fewer than from the whole list
    assert 0 < len(Gp["x"]) < len(Gw["x"]) and ctx2.read_status() == 0

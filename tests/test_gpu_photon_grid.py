"""GPU photon step on a 2D grid against the oracle: the TSC gather of the photon kernel for
photons inside, on the border of and beyond the grid, in random order and sorted by cell
(tiles whose taps span a few cells, or the whole grid), random field values; one VB + NBW
step.  FP64 to the parity bar; mixed within single-precision error of the FP64 path."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402

from test_gpu_parity import _close_lep, _ctx, _sim  # noqa: E402

TILE = 256                 # photons per block of the photon kernel
PATCH_NODES = 1024         # nodes of a compact tile box (a tile of photons close together)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-photon-grid] {msg}", flush=True)


def _tile_fits(x, y, nx, ny, dx, dy, gx0, gy0):
    """Whether each 256-photon tile's taps (node windows of both staggers, rows on the grid,
    rows padded to a power of two) fit in a box of PATCH_NODES nodes: the test covers both
    compact tiles and tiles spread over the whole grid."""
    fits = []
    for b in range(0, len(x), TILE):
        xg = np.clip((x[b:b + TILE] - gx0) / dx, -8, nx + 8)
        yg = np.clip((y[b:b + TILE] - gy0) / dy, -8, ny + 8)
        ic, jc = np.floor(xg).astype(int), np.floor(yg).astype(int)
        xl = np.clip(ic - 1, 0, nx - 3).min()
        xh = (np.clip(ic, 0, nx - 3) + 2).max()
        r0, r1 = np.maximum(jc - 1, 0), np.minimum(jc + 2, ny - 1)
        on = r0 <= r1
        if not on.any():
            fits.append(False)
            continue
        w, h = xh - xl + 1, r1[on].max() - r0[on].min() + 1
        fits.append(6 * h * (1 << int(np.ceil(np.log2(w)))) <= 6 * PATCH_NODES)
    return np.array(fits)


@pytest.mark.parametrize("nx,ny,order", [(3, 1, "random"), (7, 5, "random"), (40, 24, "random"),
                                         (200, 30, "random"), (200, 30, "by_x")])
def test_photon_step_on_grid_matches_oracle(nx, ny, order):
    _say(f"photons on a {nx}x{ny} grid, {order}")
    rng = np.random.default_rng(100 + nx + ny)
    dx, dy, gx0, gy0 = 0.7, 0.45, -1.3, 2.1
    comps = [rng.uniform(-60.0, 60.0, (ny, nx)).astype(np.float32) for _ in range(6)]
    spec_o = dict(kind=W.FIELD_GRID2D, grid=comps, nx=nx, ny=ny, dx=dx, dy=dy, gx0=gx0, gy0=gy0)
    spec_g = dict(spec_o, grid=[torch.as_tensor(c).cuda() for c in comps])
    n = 3000
    st = W.photons(n, seed=200 + nx, eps0=3000.0, eps_rel_spread=0.3, divergence=0.3, x_mean=0.0, x_sigma=1.0,
                   r_sigma=1.0, id0=0)
    st["x"] = gx0 + dx * rng.uniform(-3.0, nx + 2.0, n)
    st["y"] = gy0 + dy * rng.uniform(-3.0, ny + 2.0, n)
    if order == "by_x":
        o = np.argsort(st["x"], kind="stable")
        st = {k: v[o].copy() for k, v in st.items()}
        st["id"] = np.arange(n, dtype=np.uint64)
    fits = _tile_fits(st["x"], st["y"], nx, ny, dx, dy, gx0, gy0)
    if (1 << int(np.ceil(np.log2(nx)))) * ny <= PATCH_NODES:     # the whole grid fits
        assert fits.all()
    elif order == "random":
        assert not fits.any()
    else:
        assert fits.sum() >= len(fits) - 1
    cfg = {"dt": W.TWO_PI / 500, "procs": oracle.PROC_VB | oracle.PROC_NBW, "seed": 21, "next_id": 1 << 41}
    step = 40
    f = oracle.make_field(spec_o)
    G = oracle.PhotonArrays.from_state(st)
    em, ep = oracle.LeptonArrays.empty(n, -1), oracle.LeptonArrays.empty(n, 1)
    sim = _sim(cfg)
    sim.photon_step(f, G, em, ep, step)
    ctx = _ctx(cfg)
    Gg = Q.Photons.from_state(st)
    emg, epg = Q.Leptons(n, -1), Q.Leptons(n, 1)
    ctx.step_photons(Q.whole(spec_g), Gg, emg, epg, step)
    go = Gg.to_numpy()
    ov = G.view()
    # |E_red| at each photon (the field normal to k that sets its basis): e1 = E_red / |E_red|
    # carries the gather's rounding amplified by typical / |E_red|, so it is held to the
    # parity bar where the field is not small and to 1e-6 elsewhere
    E, B = oracle.field_eval_points(spec_o, step * cfg["dt"], np.stack([st["x"], st["y"], st["z"]], 1))
    k = np.stack([st["kx"], st["ky"], st["kz"]], 1)
    nk = k / np.linalg.norm(k, axis=1, keepdims=True)
    Er = E - np.sum(nk * E, axis=1, keepdims=True) * nk + np.cross(nk, B)
    big = np.linalg.norm(Er, axis=1) > 1.0
    assert big.sum() > 300, big.sum()
    assert len(go["x"]) == len(ov["x"])
    assert np.array_equal(go["id"], ov["id"]) and np.array_equal(go["alive"], ov["alive"])
    for q in ("x", "y", "z", "kx", "ky", "kz"):
        assert np.max(np.abs(go[q] - ov[q]) / (np.abs(ov[q]) + 1.0)) < 1e-10, q
    for q in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z"):
        d = np.abs(go[q] - ov[q])
        assert np.max(d[big]) < 1e-10 and np.max(d) < 1e-6, (q, np.max(d[big]), np.max(d))
    _close_lep(emg.to_numpy(), em.view(), what="electrons")
    _close_lep(epg.to_numpy(), ep.view(), what="positrons")
    # mixed: within single precision of the FP64 path (same draws; decisions may differ only
    # where the pair probability sits within rounding of the draw)
    ctxm = _ctx(cfg, precision=Q.QED_MIXED)
    Gm = Q.Photons.from_state(st, precision=Q.QED_MIXED)
    emm, epm = Q.Leptons(n, -1, precision=Q.QED_MIXED), Q.Leptons(n, 1, precision=Q.QED_MIXED)
    ctxm.step_photons(Q.whole(spec_g), Gm, emm, epm, step)
    gm = Gm.to_numpy()
    same = (gm["alive"] == go["alive"]) & big
    assert (gm["alive"] == go["alive"]).sum() >= n - 2
    for q in ("e1x", "e1y", "e1z", "xi1", "xi2", "xi3"):
        err = np.max(np.abs(gm[q][same].astype(np.float64) - go[q][same]))
        assert err < 2e-5, (q, err)

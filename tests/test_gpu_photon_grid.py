"""GPU photon step on a 2D grid against the oracle: the TSC gather of the photon kernel for
photons inside, on the border of and beyond the grid, in random order, sorted by x, and in
wavefront-sized clusters (the kernel's LDS box path, with live and dead outliers that send
a wavefront back to the global gather), random field values; one VB + NBW step.  FP64 to
the parity bar; mixed within single-precision error of the FP64 path."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402

from test_gpu_parity import _close_lep, _ctx, _sim  # noqa: E402

WAVE = 64                  # photons per wavefront of the photon kernel
WB_NODES = 128             # nodes per component of a wavefront's LDS box of grid nodes


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-photon-grid] {msg}", flush=True)


def _wave_box(x, y, alive, nx, ny, dx, dy, gx0, gy0, limit=WB_NODES):
    """Whether each wavefront of 64 photons takes the kernel's LDS box path: the stencil
    nodes of every live photon (either stagger) span a box of at most `limit` nodes inside
    the grid (WB_NODES; a box of 64 nodes or fewer is filled by one load per lane)."""
    res = []
    for b in range(0, len(x), WAVE):
        a = alive[b:b + WAVE] != 0
        if not a.any():
            res.append(False)
            continue
        X, Y = (x[b:b + WAVE][a] - gx0) * (1.0 / dx), (y[b:b + WAVE][a] - gy0) * (1.0 / dy)
        i0, i1 = np.floor(X).min() - 1, np.floor(X + 0.5).max() + 1
        j0, j1 = np.floor(Y).min() - 1, np.floor(Y + 0.5).max() + 1
        w, h = i1 - i0 + 1, j1 - j0 + 1
        res.append(bool(i0 >= 0 and j0 >= 0 and i1 < nx and j1 < ny and w * h <= limit))
    return np.array(res)


@pytest.mark.parametrize("nx,ny,order", [(3, 1, "random"), (7, 5, "random"), (40, 24, "random"),
                                         (200, 30, "random"), (200, 30, "by_x"), (40, 24, "clusters"),
                                         (200, 30, "clusters")])
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
    elif order == "clusters":
        # each wavefront's photons within +-2.5 nodes of a centre anywhere over the grid and
        # its border; every third wavefront has an outlier, live or dead
        nw = (n + WAVE - 1) // WAVE
        cx, cy = rng.uniform(-1.0, nx + 1.0, nw), rng.uniform(-1.0, ny + 1.0, nw)
        w = np.arange(n) // WAVE
        st["x"] = gx0 + dx * (cx[w] + rng.uniform(-2.5, 2.5, n))
        st["y"] = gy0 + dy * (cy[w] + rng.uniform(-2.5, 2.5, n))
        for b in range(0, nw, 3):
            lane = b * WAVE + int(rng.integers(0, min(WAVE, n - b * WAVE)))
            st["x"][lane] = gx0 + dx * rng.uniform(-3.0, nx + 2.0)
            st["alive"][lane] = b % 2
    fits = _wave_box(st["x"], st["y"], st["alive"], nx, ny, dx, dy, gx0, gy0)
    _say(f"{int(fits.sum())} of {len(fits)} wavefronts on the LDS box path")
    if order == "clusters":
        one = _wave_box(st["x"], st["y"], st["alive"], nx, ny, dx, dy, gx0, gy0, limit=64).sum()
        assert 0.15 * len(fits) < fits.sum() < 0.9 * len(fits)
        assert one >= 3 and fits.sum() - one >= 3          # boxes filled by one and two loads
    else:
        assert not fits.any()
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

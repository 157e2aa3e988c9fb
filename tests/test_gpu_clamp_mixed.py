"""Mixed precision beyond the top of the tables.  Leptons at chi of several thousand (the
spectrum tables end at chi = 1e3) sample photons from the last row pair of the FP32
paired-row copy, and those photons create pairs from the last row pair of the FP32 pair
spectrum.  The step must flag QED_ST_CLAMP and leave finite states: photon energies below
the largest lepton energy, spins and Stokes vectors no longer than one.  In the photon
step, total momentum is conserved: the photons that decayed hand their momentum to the
pairs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-clamp] {msg}", flush=True)


def _momentum(d, keys):
    return np.array([d[k].sum() for k in keys])


def test_mixed_steps_past_the_table_tops():
    _say("mixed, chi beyond the tables")
    n = 256
    st = W.beam(n, seed=17, gamma0=5e5, gamma_rel_spread=0.01, divergence=0.0, x_mean=0, x_sigma=0, r_sigma=0,
                spin="iso")
    spec = {"kind": W.FIELD_CONST, "e0": (0, 3e3, 0), "b0": (0, 0, -3e3)}   # chi ~ 7e3
    procs = Q.PROC_NCS | Q.PROC_NCS_STOKES | Q.PROC_NBW | Q.PROC_VB
    ctx = Q.Context(dt=0.1, procs=procs, seed=3, id_start=0, precision=Q.QED_MIXED)
    L = Q.Leptons.from_state(st, capacity=64 * n, charge=-1, precision=Q.QED_MIXED)
    G = Q.Photons(64 * n, precision=Q.QED_MIXED)
    segs = Q.whole(spec)
    for s in range(4):
        ctx.step_leptons(segs, L, G, s)
    torch.cuda.synchronize()
    assert ctx.read_status() & Q.ST_CLAMP
    g = G.to_numpy()
    assert G.count > 50, G.count
    k = np.sqrt(g["kx"] ** 2 + g["ky"] ** 2 + g["kz"] ** 2)
    gmax = np.sqrt(1 + st["px"] ** 2 + st["py"] ** 2 + st["pz"] ** 2).max()
    assert np.all(np.isfinite(k)) and np.all(k > 0) and np.all(k < gmax)
    xi = np.sqrt(g["xi1"] ** 2 + g["xi2"] ** 2 + g["xi3"] ** 2)
    assert np.all(xi <= 1 + 1e-5)
    l0 = L.to_numpy()
    assert all(np.all(np.isfinite(l0[c])) for c in ("x", "px", "py", "pz", "sx", "sy", "sz"))
    assert np.all(np.sqrt(l0["sx"] ** 2 + l0["sy"] ** 2 + l0["sz"] ** 2) <= 1 + 1e-5)
    # photon step: pairs from the last row pair of the FP32 pair spectrum
    em = Q.Leptons(64 * n, -1, precision=Q.QED_MIXED)
    ep = Q.Leptons(64 * n, 1, precision=Q.QED_MIXED)
    ktot0 = _momentum(g, ("kx", "ky", "kz"))
    ctx.step_photons(segs, G, em, ep, 4)
    torch.cuda.synchronize()
    assert ctx.read_status() & Q.ST_CLAMP
    assert em.count > 0 and em.count == ep.count
    g1, e1, p1 = G.to_numpy(), em.to_numpy(), ep.to_numpy()
    alive = g1["alive"].astype(bool)
    assert (~alive).sum() == em.count
    ktot1 = _momentum({c: g1[c][alive] for c in ("kx", "ky", "kz")}, ("kx", "ky", "kz"))
    ptot = _momentum(e1, ("px", "py", "pz")) + _momentum(p1, ("px", "py", "pz"))
    assert np.abs(ktot1 + ptot - ktot0).max() <= 1e-6 * np.abs(ktot0).max()
    for d in (e1, p1):
        assert all(np.all(np.isfinite(d[c])) for c in ("x", "px", "py", "pz", "sx", "sy", "sz"))
        assert np.all(np.sqrt(d["sx"] ** 2 + d["sy"] ** 2 + d["sz"] ** 2) <= 1 + 1e-5)

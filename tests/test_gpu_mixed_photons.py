"""The photon step in mixed precision (QED_MIXED: FP32 Stokes vector, basis, rates, CDF
sampling and pair spins; FP64 positions, momenta and event comparison) against the FP64
GPU path on the same inputs and draws (Sec. III.C.2 frame rotation, Sec. III.F
birefringence, Sec. III.D pair creation), and one mixed step against the oracle.

Bar: per photon, the Stokes vector and basis within single-precision error accumulated
over the steps; event decisions identical except where the draw falls within FP32 rounding
of the probability (a handful); for pairs present in both runs, momenta to 1e-4 and spins
along the same axis; the pair spectrum and mean pair polarisation statistically equal."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402

from test_gpu_parity import _photon_case, _sim  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-mixed-photons] {msg}", flush=True)


def _run(prec, st, spec, cfg, s0, steps):
    n = len(st["x"])
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"], precision=prec)
    G = Q.Photons.from_state(st, precision=prec)
    em, ep = Q.Leptons(n, -1, precision=prec), Q.Leptons(n, 1, precision=prec)
    segs = Q.whole(spec)
    for s in range(s0, s0 + steps):
        ctx.step_photons(segs, G, em, ep, s)
    return G.to_numpy(), em.to_numpy(), ep.to_numpy(), ctx.read_status()


def test_mixed_photon_step_tracks_fp64():
    _say("mixed vs fp64, VB + NBW, 250 steps")
    st, spec, cfg, s0, steps = _photon_case(n=20000)
    ga, ema, epa, sta = _run(Q.QED_FP64, st, spec, cfg, s0, steps)
    gb, emb, epb, stb = _run(Q.QED_MIXED, st, spec, cfg, s0, steps)
    assert sta == stb == 0, (sta, stb)
    # event decisions
    flips = int(np.sum(ga["alive"] != gb["alive"]))
    assert len(ema["x"]) > 500, len(ema["x"])
    assert flips <= 5, flips
    both = (ga["alive"] == 1) & (gb["alive"] == 1)
    for k in ("xi1", "xi2", "xi3"):
        assert np.max(np.abs(ga[k][both] - gb[k][both])) < 2e-4, k
    for k in ("e1x", "e1y", "e1z"):
        assert np.max(np.abs(ga[k][both] - gb[k][both])) < 2e-5, k
    for k in ("x", "y", "z"):
        assert np.max(np.abs(ga[k] - gb[k]) / (1 + np.abs(ga[k]))) < 1e-12, k   # FP64 in both
    # pairs present in both runs (same photon id -> same pair ids)
    for a, b, what in ((ema, emb, "electrons"), (epa, epb, "positrons")):
        assert abs(len(a["x"]) - len(b["x"])) <= 5, what
        ia = {int(v): i for i, v in enumerate(a["id"])}
        common = [(ia[int(v)], j) for j, v in enumerate(b["id"]) if int(v) in ia]
        assert len(common) >= len(a["x"]) - 5, what
        i_a, i_b = np.array([c[0] for c in common]), np.array([c[1] for c in common])
        pa = np.stack([a[k][i_a] for k in ("px", "py", "pz")])
        pb = np.stack([b[k][i_b] for k in ("px", "py", "pz")])
        rel = np.linalg.norm(pa - pb, axis=0) / np.linalg.norm(pa, axis=0)
        assert np.mean(rel < 1e-4) > 0.99, (what, np.quantile(rel, [0.5, 0.99]))
        sa = np.stack([a[k][i_a] for k in ("sx", "sy", "sz")])
        sb = np.stack([b[k][i_b] for k in ("sx", "sy", "sz")])
        dots = np.sum(sa * sb, axis=0)
        assert np.mean(dots > 0.999) > 0.98, (what, np.mean(dots > 0.999))
        # spectrum (energy share of the photon) and mean polarisation: statistically equal
        ea, eb = np.linalg.norm(pa, axis=0), np.linalg.norm(pb, axis=0)
        m = len(ea)
        assert abs(ea.mean() - eb.mean()) < 4 * ea.std() / math.sqrt(m), what
        for c in range(3):
            assert abs(sa[c].mean() - sb[c].mean()) < 4 / math.sqrt(m), (what, c)


def test_one_mixed_photon_step_against_the_oracle():
    """One mixed step from the same state and draws as the oracle's FP64 step: Stokes and
    basis to FP32 error, decisions and pair ids identical (a single step leaves no room for
    accumulated differences)."""
    _say("one mixed photon step vs oracle")
    st, spec, cfg, s0, _ = _photon_case(n=20000)
    s = 2150                          # the photons at the middle of the pulse
    n = len(st["x"])
    f = oracle.make_field(spec)
    G = oracle.PhotonArrays.from_state(st)
    em, ep = oracle.LeptonArrays.empty(n, -1), oracle.LeptonArrays.empty(n, 1)
    sim = _sim(cfg)
    sim.photon_step(f, G, em, ep, s)
    gb, emb, epb, stb = _run(Q.QED_MIXED, st, spec, cfg, s, 1)
    o = G.view()
    assert np.sum(o["alive"] != gb["alive"]) <= 1
    both = (o["alive"] == 1) & (gb["alive"] == 1)
    for k in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z"):
        assert np.max(np.abs(o[k][both] - gb[k][both])) < 2e-6, k
    for k in ("x", "y", "z"):
        assert np.max(np.abs(o[k] - gb[k]) / (1 + np.abs(o[k]))) < 1e-14, k
    assert em.count > 0
    ov = em.view()
    common = np.intersect1d(ov["id"], emb["id"])
    assert len(common) >= em.count - 1

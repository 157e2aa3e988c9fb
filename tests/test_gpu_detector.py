"""GPU parity of the detector diagnostics (qed_hist_photons / qed_hist_leptons, the
post-processing step of the VB algorithm, Sec. III.F) against the oracle on the same
particles: unit-weight counts exact, sums within 1e-12 relative (order of the
floating-point atomics aside), both precisions; binning at birth step by step equals
binning the final list when photons are not stepped; argument checks."""
import numpy as np
import pytest

import oracle
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
    print(f"[gpu-detector] {msg}", flush=True)


def _photons(n, seed=5):
    st = W.photons(n, seed=seed, eps0=300.0, eps_rel_spread=0.6, divergence=0.02, x_mean=0, x_sigma=1, r_sigma=1,
                   id0=0)
    st["kx"][:n // 50] *= -1
    st["alive"][n // 50:n // 25] = 0
    st["w"] = np.ones(n)
    for k in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z"):   # what a mixed list can hold
        st[k] = st[k].astype(np.float32).astype(np.float64)
    return st


def _compare(got, want):
    assert np.array_equal(got[..., 0], want[..., 0])
    scale = np.abs(want).max(axis=(0, 1)) + 1e-300
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want) + 1e-13 * scale)


@pytest.mark.parametrize("prec", [Q.QED_FP64, Q.QED_MIXED])
@pytest.mark.parametrize("axes,n,lo,hi", [((Q.AX_SLOPE_Y, Q.AX_SLOPE_Z), (40, 30), (-0.05, -0.04), (0.05, 0.04)),
                                          ((Q.AX_SLOPE_R, Q.AX_ENERGY), (20, 64), (0.0, 1.0), (0.06, 3.3))])
def test_photon_histogram_matches_oracle(prec, axes, n, lo, hi):
    _say(f"photons {axes} prec {prec}")
    st = _photons(50_000)
    h_o = oracle.hist_spec(axes, n, lo, hi, (0.3, 1.0, -0.2))
    h_g = Q.hist_spec(axes, n, lo, hi, (0.3, 1.0, -0.2))
    want = oracle.hist_photons(oracle.PhotonArrays.from_state(st), 1234, h_o)
    ctx = Q.Context(dt=0.01, procs=Q.PROC_NCS, seed=1, id_start=0, precision=prec)
    G = Q.Photons.from_state(st, precision=prec)
    got = ctx.hist_photons(G, 1234, h_g).cpu().numpy()
    assert want[..., 0].sum() > 20_000
    _compare(got, want)
    got2 = ctx.hist_photons(G, 1234, h_g, out=torch.as_tensor(got).cuda()).cpu().numpy()   # accumulates
    assert np.array_equal(got2[..., 0], 2 * want[..., 0])


@pytest.mark.parametrize("prec", [Q.QED_FP64, Q.QED_MIXED])
def test_lepton_histogram_matches_oracle(prec):
    _say(f"leptons prec {prec}")
    st = W.c2(30_000)["leptons"]
    if prec == Q.QED_MIXED:
        st = dict(st, **{k: st[k].astype(np.float32).astype(np.float64) for k in ("sx", "sy", "sz")})
    axes, n, lo, hi = (Q.AX_ENERGY, Q.AX_SLOPE_Y), (50, 24), (3.0, -3e-3), (3.6, 3e-3)
    want = oracle.hist_leptons(oracle.LeptonArrays.from_state(st), 0, oracle.hist_spec(axes, n, lo, hi))
    ctx = Q.Context(dt=0.01, procs=Q.PROC_NCS, seed=1, id_start=0, precision=prec)
    got = ctx.hist_leptons(Q.Leptons.from_state(st, precision=prec), 0, Q.hist_spec(axes, n, lo, hi)).cpu().numpy()
    assert want[..., 0].sum() > 20_000
    _compare(got, want)


def test_binning_at_birth_equals_binning_the_final_list():
    """NCS only (photons are not stepped): the sum of per-step histograms of the newborn
    photons is the histogram of the final photon list."""
    _say("at birth")
    cfg = W.c2(20_000, start_step=2450)
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                    precision=Q.QED_MIXED)
    L = Q.Leptons.from_state(cfg["leptons"], precision=Q.QED_MIXED)
    G = Q.Photons(400_000, precision=Q.QED_MIXED)
    h = Q.hist_spec((Q.AX_SLOPE_Y, Q.AX_ENERGY), (32, 48), (-0.03, 0.0), (0.03, 3.4), (0, 1, 0))
    acc = torch.zeros((48, 32, 5), dtype=torch.float64, device="cuda")
    segs = Q.whole(cfg["field"])
    for s in range(2450, 2500):
        before = G.count
        ctx.step_leptons(segs, L, G, s)
        ctx.hist_photons(G, before, h, out=acc)
    full = ctx.hist_photons(G, 0, h).cpu().numpy()
    a = acc.cpu().numpy()
    assert G.count > 5000 and full[..., 0].sum() > 0.5 * G.count
    assert np.array_equal(a[..., 0], full[..., 0])
    assert np.allclose(a, full, rtol=1e-12, atol=1e-9)


def test_histogram_arguments_are_checked():
    ctx = Q.Context(dt=0.01, procs=Q.PROC_NCS, seed=1, id_start=0)
    G = Q.Photons.from_state(_photons(100))
    out = torch.zeros((4, 4, 5), dtype=torch.float64, device="cuda")
    for bad in (Q.hist_spec((Q.AX_ENERGY, Q.AX_ENERGY), (4, 4), (0, 0), (1, 1)),
                Q.hist_spec((Q.AX_SLOPE_Y, Q.AX_ENERGY), (4, 300), (0, 0), (1, 1)),
                Q.hist_spec((Q.AX_SLOPE_Y, Q.AX_SLOPE_Z), (4, 4), (1, 0), (1, 1)),
                Q.hist_spec((Q.AX_SLOPE_Y, 9), (4, 4), (0, 0), (1, 1)),
                Q.hist_spec((Q.AX_SLOPE_Y, Q.AX_SLOPE_Z), (4, 4), (0, 0), (1, 1), (0, 0, 0))):
        with pytest.raises(Q.QedError):
            ctx.hist_photons(G, 0, bad, out=out)

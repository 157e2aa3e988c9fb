"""Checkpoint / resume: the particle lists, the step index and the context's id counter are
the whole state of a run (Philox is keyed by (id, step); the tables are rebuilt the same
way).  A run stopped halfway, its lists copied to the host, and continued in a fresh
context from those copies and the saved id counter equals the uninterrupted run bit for
bit: electrons, positrons and photons (NCS with photon Stokes, NBW pairs, birefringence)."""
import math

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
    print(f"[gpu-resume] {msg}", flush=True)


PROCS = Q.PROC_NCS | Q.PROC_NCS_STOKES | Q.PROC_NBW | Q.PROC_VB
FIELD = {"kind": Q.FIELD_PW, "circular": 0, "a0": 300.0, "ncycles": 8.0, "phase0": 0.0, "pol_angle": 0.0,
         "phi_start": 0.0}
DT = 2 * math.pi / 500


def _fresh(prec, id_start, st_em, st_ep=None, st_g=None):
    ctx = Q.Context(dt=DT, procs=PROCS, seed=7, id_start=id_start, precision=prec)
    n = len(st_em["x"])
    em = Q.Leptons.from_state(st_em, capacity=4 * n, charge=-1, precision=prec)
    ep = Q.Leptons.from_state(st_ep, capacity=4 * n, charge=1, precision=prec) if st_ep and len(st_ep["x"]) \
        else Q.Leptons(4 * n, 1, precision=prec)
    G = Q.Photons.from_state(st_g, capacity=40 * n, precision=prec) if st_g and len(st_g["x"]) \
        else Q.Photons(40 * n, precision=prec)
    return ctx, em, ep, G


def _run(ctx, em, ep, G, steps):
    segs = Q.whole(FIELD)
    for s in steps:
        ctx.step(segs, em, ep, G, s)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [Q.QED_FP64, Q.QED_MIXED], ids=["fp64", "mixed"])
def test_resume_from_host_copies_is_bitwise(prec):
    _say(f"resume {prec}")
    st = W.beam(3000, seed=41, gamma0=4000.0, gamma_rel_spread=0.05, divergence=1e-3, x_mean=8 * math.pi,
                x_sigma=math.pi, r_sigma=2 * math.pi, spin="iso")
    id0 = 1 << 40
    ctx, em, ep, G = _fresh(prec, id0, st)
    _run(ctx, em, ep, G, range(0, 60))
    whole = (em.to_numpy(), ep.to_numpy(), G.to_numpy(), ctx.next_id())
    del ctx, em, ep, G
    ctx, em, ep, G = _fresh(prec, id0, st)
    _run(ctx, em, ep, G, range(0, 30))
    saved = (em.to_numpy(), ep.to_numpy(), G.to_numpy(), ctx.next_id())   # the checkpoint
    del ctx, em, ep, G
    ctx, em, ep, G = _fresh(prec, saved[3], saved[0], saved[1], saved[2])
    _run(ctx, em, ep, G, range(30, 60))
    resumed = (em.to_numpy(), ep.to_numpy(), G.to_numpy(), ctx.next_id())
    assert len(whole[1]["x"]) > 0 and len(whole[2]["x"]) > 100      # pairs and photons happened
    for a, b, what in zip(whole[:3], resumed[:3], ("electrons", "positrons", "photons")):
        assert a.keys() == b.keys()
        for k in a:
            assert np.array_equal(a[k], b[k]), (what, k)
    assert whole[3] == resumed[3]

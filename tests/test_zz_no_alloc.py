"""The allocation-free lepton step (qed_step_leptons_noalloc) against qed_step_leptons: the
same kernels with their work memory in the library's fixed device array instead of
context-owned buffers, so every lepton, photon, id and count must be bit for bit the same.
Two calls in a row on the same GPU, the second with a smaller list (the array keeps the
first call's contents), both precisions; sizes past the array's limit are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402
import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _run(prec, st, cfg, noalloc, steps):
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"], precision=prec)
    L = Q.Leptons.from_state(st, precision=prec)
    G = Q.Photons(len(st["x"]), precision=prec)
    segs = Q.whole(cfg["field"])
    for s in steps:
        if noalloc:
            ctx.step_leptons_noalloc(segs, L, G, s)
        else:
            ctx.step_leptons(segs, L, G, s)
    out = (L.to_numpy(), G.to_numpy(), ctx.next_id(), ctx.read_status())
    ctx.close()
    return out


@pytest.mark.parametrize("prec", [Q.QED_MIXED, Q.QED_FP64])
def test_noalloc_step_equals_the_step(prec):
    cfg = W.c2(300_000, start_step=2450)
    for n, steps in ((300_000, range(2450, 2454)), (70_001, range(2460, 2463))):
        print(f"[no-alloc] precision {prec}, {n} leptons, steps {steps.start}..{steps.stop - 1}", flush=True)
        st = {k: v[:n].copy() for k, v in cfg["leptons"].items()}
        ref = _run(prec, st, cfg, False, steps)
        got = _run(prec, st, cfg, True, steps)
        assert len(ref[1]["x"]) > 1000
        for a, b in ((ref[0], got[0]), (ref[1], got[1])):
            assert a.keys() == b.keys()
            for k in a:
                assert np.array_equal(a[k], b[k]), (n, k)
        assert ref[2:] == got[2:]


def test_noalloc_limits():
    cfg = W.c2(1000, start_step=2450)
    ctx = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"])
    big = Q.Leptons(Q.NOALLOC_MAX_LEPTONS + 1, -1)
    with pytest.raises(Q.QedError) as e:
        ctx.step_leptons_noalloc(Q.whole(cfg["field"]), big, None, 0)
    assert "limit" in str(e.value)
    two = Q.segments([(0, 10, cfg["field"]), (10, 20, cfg["field"])])
    small = Q.Leptons(100, -1)
    with pytest.raises(Q.QedError):
        ctx.step_leptons_noalloc(two, small, None, 0)
    ctx.close()

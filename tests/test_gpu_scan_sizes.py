"""Ordered stream compaction of photon lists whose tile count passes the scan kernel's
register path.  Each of the scan's 1024 threads keeps the first 8 counts of its run in
registers between its two passes; past 8192 tiles of 256 photons a run is longer and the
rest is read again.  For lists just at, just past and well past that size, the compacted
list must hold the alive photons in index order, every array bit for bit, with an exact
count.  The expected result is numpy's boolean selection, which is the plain definition
of a stable compaction."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-scan] {msg}", flush=True)


def _photon_state(n, seed, alive_frac):
    g = np.random.default_rng(seed)
    st = {k: g.standard_normal(n) for k in Q.PHOTON_KEYS}
    st["id"] = g.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    st["alive"] = (g.random(n) < alive_frac).astype(np.uint8)
    return st


@pytest.mark.parametrize("n,prec", [(8192 * 256, Q.QED_FP64), (8192 * 256 + 1, Q.QED_FP64),
                                    (3_000_077, Q.QED_FP64), (3_000_077, Q.QED_MIXED)],
                         ids=["8192-tiles", "8192-tiles+1", "11719-tiles", "11719-tiles-mixed"])
def test_compaction_past_the_register_path(n, prec):
    _say(f"compact n={n} prec={prec}")
    st = _photon_state(n, seed=n % 1000 + prec, alive_frac=0.61)
    keep = st["alive"].astype(bool)
    src = Q.Photons.from_state(st, precision=prec)
    dst = Q.Photons(n, precision=prec)
    ctx = Q.Context(dt=0.01, procs=Q.PROC_VB, seed=1, id_start=0, precision=prec)
    ctx.compact_photons(src, dst)
    torch.cuda.synchronize()
    got = dst.to_numpy()
    assert dst.count == int(keep.sum())
    low = np.float32 if prec == Q.QED_MIXED else np.float64
    for k in Q.PHOTON_KEYS:
        want = st[k][keep]
        if k.startswith("xi") or k.startswith("e1"):
            want = want.astype(low).astype(np.float64)
        assert np.array_equal(got[k], want), k
    assert np.array_equal(got["id"], st["id"][keep])
    assert np.all(got["alive"] == 1)
    assert ctx.read_status() & Q.ST_OVERFLOW == 0

"""GPU tests of the batched step (many collisions as segments of one list), of step
loops captured in a hipGraph and replayed with a device step counter, and of the launch
shapes the autotuner chooses from.

Bar: graph replay == eager calls and every launch shape == every other, bitwise (same
draws, same order, same ids).  Batched == one collision at a time with identical ids,
order and counts and values to rounding: the batched launch reads each segment's field
kind at run time while a single-collision launch is specialised on it, and the compiler
may contract the field arithmetic differently in the two (1e-12 in FP64; FP32 rounding
in mixed mode).  A batched sample of the collisions against the FP64 oracle to 1e-10.
"""
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
    print(f"[gpu-batching] {msg}", flush=True)


def _cfg(n_collisions=64, n_min=100, n_max=3000, start_step=0):
    return W.c4(n_collisions, n_min=n_min, n_max=n_max, start_step=start_step)


def _ctx(cfg, precision):
    return Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                     precision=precision)


def _batched(cfg, precision, steps, tuning=None, photon_cap=None):
    ctx = _ctx(cfg, precision)
    if tuning is not None:
        ctx.set_tuning(**tuning)
    L = Q.Leptons.from_state(cfg["leptons"], precision=precision)
    G = Q.Photons(photon_cap or len(cfg["leptons"]["x"]) * 2, precision=precision)
    segs = Q.segments(cfg["segments"])
    for s in steps:
        ctx.step_leptons(segs, L, G, s)
    torch.cuda.synchronize()
    return ctx, L.to_numpy(), G.to_numpy()


def _same(a: dict, b: dict, what: str):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("precision", [Q.QED_FP64, Q.QED_MIXED], ids=["fp64", "mixed"])
def test_batched_equals_one_by_one(precision):
    """64 collisions in one list (one launch per step) against the same collisions as 64
    lists stepped one after the other into one photon list."""
    _say(f"batched vs one-by-one {precision}")
    cfg = _cfg()
    steps = range(0, 25)
    ctx_b, Lb, Gb = _batched(cfg, precision, steps)
    ctx = _ctx(cfg, precision)
    lists, specs = [], []
    for (b, e, spec) in cfg["segments"]:
        lists.append(Q.Leptons.from_state({k: v[b:e] for k, v in cfg["leptons"].items()}, precision=precision))
        specs.append(Q.whole(spec))
    G = Q.Photons(len(cfg["leptons"]["x"]) * 2, precision=precision)
    for s in steps:
        for L, sg in zip(lists, specs):
            ctx.step_leptons(sg, L, G, s)
    torch.cuda.synchronize()
    one = {k: np.concatenate([L.to_numpy()[k] for L in lists]) for k in Lb}
    go = G.to_numpy()
    assert np.array_equal(Lb["id"], one["id"]) and np.array_equal(Gb["id"], go["id"])
    assert len(Gb["x"]) == len(go["x"]) > 200
    assert ctx_b.next_id() == ctx.next_id()
    tol, stol = (1e-12, 1e-12) if precision == Q.QED_FP64 else (1e-8, 2e-5)
    pm = np.sqrt(one["px"] ** 2 + one["py"] ** 2 + one["pz"] ** 2) + 1.0
    xm = np.sqrt(one["x"] ** 2 + one["y"] ** 2 + one["z"] ** 2) + 1.0
    for k in ("px", "py", "pz"):
        assert np.max(np.abs(Lb[k] - one[k]) / pm) < tol, k
    for k in ("x", "y", "z"):
        assert np.max(np.abs(Lb[k] - one[k]) / xm) < tol, k
    for k in ("sx", "sy", "sz"):
        assert np.max(np.abs(Lb[k] - one[k])) < stol, k
    km = np.sqrt(go["kx"] ** 2 + go["ky"] ** 2 + go["kz"] ** 2) + 1.0
    for k in ("kx", "ky", "kz"):
        assert np.max(np.abs(Gb[k] - go[k]) / km) < tol, k
    for k in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z"):
        assert np.max(np.abs(Gb[k] - go[k])) < stol, k


def test_batched_sample_vs_oracle_fp64():
    """Eight of the collisions (LP and CP, random polarisation angles) against the oracle."""
    _say("batched vs oracle")
    cfg = _cfg(n_collisions=8, n_min=100, n_max=600)
    steps = range(0, 40)
    _, Lb, Gb = _batched(cfg, Q.QED_FP64, steps)
    sim = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], next_id=cfg["next_id"])
    G = oracle.PhotonArrays.empty(len(cfg["leptons"]["x"]) * 2)
    Ls, fs = [], []
    for (b, e, spec) in cfg["segments"]:
        Ls.append(oracle.LeptonArrays.from_state({k: v[b:e].copy() for k, v in cfg["leptons"].items()}))
        fs.append(oracle.make_field(spec))
    for s in steps:
        for L, f in zip(Ls, fs):
            sim.step(f, L, None, G, s)
    ov = {k: np.concatenate([L.view()[k] for L in Ls]) for k in Ls[0].view()}
    assert np.array_equal(Lb["id"], ov["id"])
    pm = np.sqrt(ov["px"] ** 2 + ov["py"] ** 2 + ov["pz"] ** 2) + 1.0
    for k in ("px", "py", "pz"):
        assert np.max(np.abs(Lb[k] - ov[k]) / pm) < 1e-10, k
    for k in ("sx", "sy", "sz"):
        assert np.max(np.abs(Lb[k] - ov[k])) < 1e-10, k
    go = G.view()
    assert len(go["x"]) == len(Gb["x"]) > 20
    assert np.array_equal(go["id"], Gb["id"])
    km = np.sqrt(go["kx"] ** 2 + go["ky"] ** 2 + go["kz"] ** 2) + 1.0
    for k in ("kx", "ky", "kz"):
        assert np.max(np.abs(Gb[k] - go[k]) / km) < 1e-10, k
    for k in ("xi1", "xi2", "xi3"):
        assert np.max(np.abs(Gb[k] - go[k])) < 1e-10, k


@pytest.mark.parametrize("kinds", ["mixed", "common"])
def test_mixed_kinds_and_gaps_vs_oracle_fp64(kinds):
    """Segments with gaps between them, boundaries inside wavefronts; particles in a gap see
    no field.  mixed: segments of different field kinds (plane waves, Gaussian beams, a
    constant field), the generic many-kind kernel and the waterfall over segments.  common:
    plane waves only, the kernel specialised on their kind, whose tiles inside one segment or
    one gap take the straight-line path and whose tiles across a boundary or a gap edge take
    a launch of their own; the first collision and the third are whole gaps (tiles with no
    segment at all).  Against the oracle, which steps the segments and the gaps as separate
    lists in index order."""
    _say(f"{kinds} kinds and gaps vs oracle")
    cfg = _cfg(n_collisions=6, n_min=150, n_max=500) if kinds == "mixed" else \
        _cfg(n_collisions=6, n_min=600, n_max=900)
    segs, pieces, prev = [], [], 0
    for k, (b, e, spec) in enumerate(cfg["segments"]):
        spec = dict(spec)
        if kinds == "common":
            if k in (0, 2):
                continue                                       # a whole collision as a gap
        elif k % 3 == 1:
            spec.update(kind=W.FIELD_GAUSS, w0=12.0, x_focus=0.0, phi_start=0.0)
        elif k % 3 == 2 and k == 2:
            spec = {"kind": W.FIELD_CONST, "e0": (0.0, 30.0, 0.0), "b0": (0.0, 0.0, -30.0)}
        lo, hi = b + 7 + 3 * k, e - 5                         # gaps at both ends
        if lo > prev:
            pieces.append((prev, lo, {"kind": W.FIELD_NONE}))
        pieces.append((lo, hi, spec))
        segs.append((lo, hi, spec))
        prev = hi
    n = len(cfg["leptons"]["x"])
    if prev < n:
        pieces.append((prev, n, {"kind": W.FIELD_NONE}))
    steps = range(0, 30)
    ctx = _ctx(cfg, Q.QED_FP64)
    L = Q.Leptons.from_state(cfg["leptons"], precision=Q.QED_FP64)
    G = Q.Photons(n * 2, precision=Q.QED_FP64)
    sg = Q.segments(segs)
    for s in steps:
        ctx.step_leptons(sg, L, G, s)
    torch.cuda.synchronize()
    Lb, Gb = L.to_numpy(), G.to_numpy()
    sim = oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], next_id=cfg["next_id"])
    Go = oracle.PhotonArrays.empty(n * 2)
    Ls = [(oracle.LeptonArrays.from_state({k: v[b:e].copy() for k, v in cfg["leptons"].items()}),
           oracle.make_field(spec)) for (b, e, spec) in pieces]
    for s in steps:
        for Lo, f in Ls:
            sim.step(f, Lo, None, Go, s)
    ov = {k: np.concatenate([Lo.view()[k] for Lo, _ in Ls]) for k in Ls[0][0].view()}
    assert np.array_equal(Lb["id"], ov["id"])
    pm = np.sqrt(ov["px"] ** 2 + ov["py"] ** 2 + ov["pz"] ** 2) + 1.0
    for k in ("px", "py", "pz"):
        assert np.max(np.abs(Lb[k] - ov[k]) / pm) < 1e-10, k
    for k in ("sx", "sy", "sz"):
        assert np.max(np.abs(Lb[k] - ov[k])) < 1e-10, k
    go = Go.view()
    assert len(go["x"]) == len(Gb["x"]) > 20
    assert np.array_equal(go["id"], Gb["id"])
    # gap particles moved on straight lines (no field): p unchanged
    p0 = cfg["leptons"]
    for (b, e, spec) in pieces:
        if spec["kind"] == W.FIELD_NONE:
            assert np.array_equal(Lb["px"][b:e], p0["px"][b:e])


def test_graph_replay_equals_eager():
    """K steps captured once (step calls + device step counter advance) and replayed R
    times, with eager work and synchronisations between the replays, equal R*K eager steps;
    every replay is checked."""
    _say("graph replay")
    cfg = _cfg(n_collisions=16)
    K, R, s0 = 6, 3, 5
    prec = Q.QED_MIXED
    # eager reference, checked after each block of K steps
    ctx_e = _ctx(cfg, prec)
    Le = Q.Leptons.from_state(cfg["leptons"], precision=prec)
    Ge = Q.Photons(len(cfg["leptons"]["x"]) * 2, precision=prec)
    segs_e = Q.segments(cfg["segments"])
    ref = []
    ctx_e.step_leptons(segs_e, Le, Ge, s0 - 1)
    for r in range(R):
        for k in range(K):
            ctx_e.step_leptons(segs_e, Le, Ge, s0 + r * K + k)
        torch.cuda.synchronize()
        ref.append((Le.to_numpy(), Ge.to_numpy(), ctx_e.next_id()))
    # graph
    ctx = _ctx(cfg, prec)
    L = Q.Leptons.from_state(cfg["leptons"], precision=prec)
    G = Q.Photons(len(cfg["leptons"]["x"]) * 2, precision=prec)
    segs = Q.segments(cfg["segments"])
    ctx.step_leptons(segs, L, G, s0 - 1)   # eager: sizes the staging area, uploads the segments
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ctx.set_step_counter(counter)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for k in range(K):
            ctx.step_leptons(segs, L, G, s0)
            ctx.advance_step(1)
    torch.cuda.synchronize()
    for r in range(R):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        lr, gr, ir = ref[r]
        _same(L.to_numpy(), lr, f"leptons replay {r}")
        _same(G.to_numpy(), gr, f"photons replay {r}")
        assert ctx.next_id() == ir
        assert int(counter.item()) == (r + 1) * K
    ctx.set_step_counter(None)


TUNINGS = [dict(blocks_per_cu=0, rate_lds=0, ev_group=8), dict(blocks_per_cu=2, rate_lds=1, ev_group=4),
           dict(blocks_per_cu=4, rate_lds=0, ev_group=16), dict(blocks_per_cu=8, rate_lds=1, ev_group=8),
           dict(blocks_per_cu=1, rate_lds=1, ev_group=16)]


@pytest.mark.parametrize("precision", [Q.QED_FP64, Q.QED_MIXED], ids=["fp64", "mixed"])
def test_launch_shapes_bitwise_identical(precision):
    _say(f"launch shapes {precision}")
    cfg = _cfg(n_collisions=32)
    steps = range(0, 12)
    base = None
    for t in TUNINGS:
        ctx, Lr, Gr = _batched(cfg, precision, steps, tuning=t)
        assert ctx.get_tuning() == t
        if base is None:
            base = (Lr, Gr, ctx.next_id())
        else:
            _same(Lr, base[0], f"leptons {t}")
            _same(Gr, base[1], f"photons {t}")
            assert ctx.next_id() == base[2]


def test_autotune_leaves_state_and_results_unchanged():
    _say("autotune")
    cfg = _cfg(n_collisions=32)
    prec = Q.QED_MIXED
    ctx = _ctx(cfg, prec)
    L = Q.Leptons.from_state(cfg["leptons"], precision=prec)
    G = Q.Photons(len(cfg["leptons"]["x"]) * 2, precision=prec)
    segs = Q.segments(cfg["segments"])
    before = L.to_numpy()
    id_before = ctx.next_id()
    chosen = ctx.autotune(segs, L, 0, reps=2)
    assert chosen["blocks_per_cu"] in (0, 2, 4, 8) and chosen["rate_lds"] in (0, 1) and chosen["ev_group"] in (4, 8, 16)
    assert ctx.get_tuning() == chosen
    _same(L.to_numpy(), before, "leptons after autotune")
    assert ctx.next_id() == id_before
    assert ctx.read_status() == 0
    for s in range(0, 12):
        ctx.step_leptons(segs, L, G, s)
    torch.cuda.synchronize()
    _, Lr, Gr = _batched(cfg, prec, range(0, 12))
    _same(L.to_numpy(), Lr, "leptons")
    _same(G.to_numpy(), Gr, "photons")


def test_tuning_rejects_bad_values():
    cfg = _cfg(n_collisions=2)
    ctx = _ctx(cfg, Q.QED_MIXED)
    for bad in (dict(blocks_per_cu=-1), dict(rate_lds=2), dict(ev_group=5)):
        with pytest.raises(Q.QedError):
            ctx.set_tuning(**bad)
    with pytest.raises(Q.QedError):
        ctx.advance_step(1)   # no counter registered

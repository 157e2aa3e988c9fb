"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on identical seeded
inputs.

Bar (FP64 contexts): tables to 1e-12; positions, momenta, spins, Stokes vectors and bases
within 1e-10 relative; event decisions, appended-particle order, ids and counts identical.
Mixed contexts: per particle within single-precision error of the FP64 path.
"""
import math

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
    Q.lib()   # a GPU machine without the built library is a failure, not a skip


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


# ----------------------------------------------------------------------------- helpers
def _sub(st: dict, n: int) -> dict:
    return {k: v[:n].copy() for k, v in st.items()}


def _ctx(cfg, precision=Q.QED_FP64, **kw):
    return Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                     precision=precision, p_max=kw.get("p_max", 0.1))


def _sim(cfg):
    return oracle.Sim(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], next_id=cfg["next_id"])


def _close_lep(g: dict, o: dict, tol=1e-10, what=""):
    assert len(g["x"]) == len(o["x"]), what
    assert np.array_equal(g["id"], o["id"]), what
    pmag = np.sqrt(o["px"] ** 2 + o["py"] ** 2 + o["pz"] ** 2) + 1.0
    xmag = np.sqrt(o["x"] ** 2 + o["y"] ** 2 + o["z"] ** 2) + 1.0
    for k in ("px", "py", "pz"):
        err = np.max(np.abs(g[k] - o[k]) / pmag, initial=0)
        assert err < tol, (what, k, err)
    for k in ("x", "y", "z"):
        err = np.max(np.abs(g[k] - o[k]) / xmag, initial=0)
        assert err < tol, (what, k, err)
    for k in ("sx", "sy", "sz", "w"):
        err = np.max(np.abs(g[k] - o[k]), initial=0)
        assert err < tol, (what, k, err)


def _close_pho(g: dict, o: dict, tol=1e-10, what=""):
    assert len(g["x"]) == len(o["x"]), (what, len(g["x"]), len(o["x"]))
    assert np.array_equal(g["id"], o["id"]), what
    assert np.array_equal(g["alive"], o["alive"]), what
    kmag = np.sqrt(o["kx"] ** 2 + o["ky"] ** 2 + o["kz"] ** 2) + 1.0
    xmag = np.sqrt(o["x"] ** 2 + o["y"] ** 2 + o["z"] ** 2) + 1.0
    for k in ("kx", "ky", "kz"):
        assert np.max(np.abs(g[k] - o[k]) / kmag, initial=0) < tol, (what, k)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(g[k] - o[k]) / xmag, initial=0) < tol, (what, k)
    for k in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z", "w"):
        assert np.max(np.abs(g[k] - o[k]), initial=0) < tol, (what, k, np.max(np.abs(g[k] - o[k]), initial=0))


def _oracle_photons(G: oracle.PhotonArrays) -> dict:
    return G.view()


# ----------------------------------------------------------------------------- tables
def test_tables_match_oracle():
    _say("tables")
    ctx = Q.Context(dt=0.01, procs=15, seed=1, id_start=0)
    T = oracle.tables()
    for which in range(7):
        g, o = ctx.table_export(which), T.export(which)
        err = np.abs(g - o)
        bound = 1e-12 * np.abs(o) + 1e-14 * np.abs(o).max()
        assert np.all(err <= bound), (which, np.max(err / (np.abs(o) + 1e-300)))


# ----------------------------------------------------------------------------- leptons
def _run_leptons(cfg, n, steps, mode="fused", cap_factor=3):
    st = _sub(cfg["leptons"], n)
    s0 = cfg.get("start_step", 0)
    # oracle
    f = oracle.make_field(cfg["field"])
    L = oracle.LeptonArrays.from_state(st, charge=-1)
    G = oracle.PhotonArrays.empty(cap_factor * n + 16)
    sim = _sim(cfg)
    for s in range(s0, s0 + steps):
        sim.step(f, L, None, G, s)
    # gpu
    ctx = _ctx(cfg)
    Lg = Q.Leptons.from_state(st, charge=-1)
    Gg = Q.Photons(cap_factor * n + 16)
    segs = Q.whole(cfg["field"])
    E6 = torch.zeros(6 * n, dtype=torch.float64, device="cuda")
    for s in range(s0, s0 + steps):
        if mode == "fused":
            ctx.step_leptons(segs, Lg, Gg, s)
        else:
            ctx.gather(segs, Lg, E6, s)
            ctx.push_spin(segs, Lg, s, E6=E6)
            ctx.emit(segs, Lg, E6, Gg, s)
    torch.cuda.synchronize()
    return L, G, sim, Lg, Gg, ctx


@pytest.mark.parametrize("mode", ["fused", "split"])
def test_c1_plane_wave_lp_fp64(mode):
    _say(f"c1 plane wave LP fp64 {mode}")
    cfg = W.c1(4000, start_step=400)
    L, G, sim, Lg, Gg, ctx = _run_leptons(cfg, 4000, 400, mode)
    assert G.count > 1000
    _close_lep(Lg.to_numpy(), L.view(), what="leptons")
    _close_pho(Gg.to_numpy(), _oracle_photons(G), what="photons")
    assert ctx.next_id() == sim.next_id
    assert ctx.read_status() == sim.status


def test_c1_full_length_fp64():
    """The plane-wave workload in full: 1e4 electrons through all 3000 steps (the whole
    8-cycle pulse and the free flight after it), FP64 GPU against the oracle to 1e-10 with
    identical event decisions, photon order and ids."""
    _say("c1 full length: 1e4 electrons x 3000 steps")
    cfg = W.c1(10000, start_step=0)
    L, G, sim, Lg, Gg, ctx = _run_leptons(cfg, 10000, cfg["steps"], "fused", cap_factor=8)
    assert G.count > 10000, G.count
    _close_lep(Lg.to_numpy(), L.view(), what="leptons")
    _close_pho(Gg.to_numpy(), _oracle_photons(G), what="photons")
    assert ctx.next_id() == sim.next_id
    assert ctx.read_status() == sim.status == 0


def test_c2_focused_cp_stokes_fp64():
    _say("c2 focused CP fp64 with Stokes")
    cfg = W.c2(3000, start_step=2300)
    L, G, sim, Lg, Gg, ctx = _run_leptons(cfg, 3000, 300)
    assert G.count > 300
    _close_lep(Lg.to_numpy(), L.view(), what="leptons")
    _close_pho(Gg.to_numpy(), _oracle_photons(G), what="photons")
    assert ctx.next_id() == sim.next_id


@pytest.mark.parametrize("n", [0, 1, 255, 257, 1000])
def test_ragged_and_empty_sizes(n):
    _say(f"ragged n={n}")
    cfg = W.c1(max(n, 1), start_step=600)
    cfg["leptons"] = _sub(cfg["leptons"], n)
    L, G, sim, Lg, Gg, ctx = _run_leptons(cfg, n, 40) if n > 0 else (None, None, None, None, None, None)
    if n == 0:
        ctx = _ctx(cfg)
        Lg = Q.Leptons(16, -1)
        Gg = Q.Photons(16)
        ctx.step_leptons(Q.whole(cfg["field"]), Lg, Gg, 0)
        assert Lg.count == 0 and Gg.count == 0 and ctx.next_id() == cfg["next_id"]
        return
    _close_lep(Lg.to_numpy(), L.view(), what="leptons")
    _close_pho(Gg.to_numpy(), _oracle_photons(G), what="photons")


def test_append_overflow_drops_and_flags():
    _say("overflow")
    cfg = W.c1(2000, start_step=600)
    L, G, sim, Lg, Gg, ctx = _run_leptons(cfg, 2000, 30, cap_factor=0)   # capacity 16
    assert Gg.count == 16 and G.count == 16
    assert ctx.read_status() & Q.ST_OVERFLOW and sim.status & oracle.ST_OVERFLOW
    assert ctx.next_id() == sim.next_id          # ids still consumed
    _close_pho(Gg.to_numpy(), _oracle_photons(G), what="photons")
    _close_lep(Lg.to_numpy(), L.view(), what="leptons")


def test_status_bits_pmax_clamp_nan():
    _say("status bits")
    n = 64
    st = W.beam(n, seed=5, gamma0=5e5, gamma_rel_spread=0.0, divergence=0.0, x_mean=0, x_sigma=0, r_sigma=0)
    spec = {"kind": W.FIELD_CONST, "e0": (0, 3e3, 0), "b0": (0, 0, -3e3)}   # chi ~ 7e3 > table range
    ctx = Q.Context(dt=1.0, procs=1, seed=1, id_start=0, p_max=0.05)
    Lg = Q.Leptons.from_state(st)
    ctx.step_leptons(Q.whole(spec), Lg, None, 0)
    s = ctx.read_status()
    assert s & Q.ST_PMAX and s & Q.ST_CLAMP
    # a NaN in a grid field poisons the push
    g = [torch.zeros(8, 8, dtype=torch.float32, device="cuda") for _ in range(6)]
    g[1][:] = float("nan")
    gspec = {"kind": W.FIELD_GRID2D, "grid": g, "nx": 8, "ny": 8, "dx": 1.0, "dy": 1.0, "gx0": -4.0, "gy0": -4.0}
    st2 = W.beam(4, seed=6, gamma0=10.0, gamma_rel_spread=0.0, divergence=0.0, x_mean=0, x_sigma=0.1, r_sigma=0.1)
    ctx2 = Q.Context(dt=0.1, procs=0, seed=1, id_start=0)
    L2 = Q.Leptons.from_state(st2)
    ctx2.push_spin(Q.whole(gspec), L2, 0)
    assert ctx2.read_status() & Q.ST_NAN
    ctx2.clear_status()
    assert ctx2.read_status() == 0


def test_status_bit_pair_member_below_rest_mass():
    """Photons of 2.5 m c^2 in a crossed field strong enough that pair creation is certain
    within the step: an uneven energy split leaves one member below m c^2 (momentum zero,
    QED_ST_EPS_LT1) and the pair energies still add up to the photon's."""
    _say("eps < 1")
    n = 400
    st = W.photons(n, seed=8, eps0=2.5, eps_rel_spread=0.0, divergence=0.0, x_mean=0, x_sigma=0.1, r_sigma=0.1,
                   id0=0)
    spec = {"kind": W.FIELD_CONST, "e0": (0, 8.2e4, 0), "b0": (0, 0, -8.2e4)}   # chi_gamma ~ 1
    ctx = Q.Context(dt=0.05, procs=Q.PROC_NBW, seed=3, id_start=1 << 40, p_max=10.0)
    G = Q.Photons.from_state(st)
    em, ep = Q.Leptons(n, -1), Q.Leptons(n, 1)
    ctx.step_photons(Q.whole(spec), G, em, ep, 0)
    assert ctx.read_status() & Q.ST_EPS_LT1
    assert em.count == ep.count > n // 2
    e, p = em.to_numpy(), ep.to_numpy()
    ge = np.sqrt(1 + e["px"] ** 2 + e["py"] ** 2 + e["pz"] ** 2)
    gp = np.sqrt(1 + p["px"] ** 2 + p["py"] ** 2 + p["pz"] ** 2)
    assert np.any(ge == 1.0) or np.any(gp == 1.0)                      # a member clamped at rest


def test_bitwise_repeatable():
    """The ordered append makes two runs bit-identical (race detector for the scan)."""
    _say("repeatability")
    cfg = W.c1(50000, start_step=550)
    outs = []
    for _ in range(2):
        ctx = _ctx(cfg)
        Lg = Q.Leptons.from_state(cfg["leptons"])
        Gg = Q.Photons(200000)
        segs = Q.whole(cfg["field"])
        for s in range(550, 610):
            ctx.step_leptons(segs, Lg, Gg, s)
        outs.append((Lg.to_numpy(), Gg.to_numpy()))
    for a, b in zip(outs[0], outs[1]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    assert len(outs[0][1]["x"]) > 1000


# ----------------------------------------------------------------------------- photons
def _photon_case(n=4000, steps=250, procs=oracle.PROC_VB | oracle.PROC_NBW):
    st = W.photons(n, seed=44, eps0=3000.0, eps_rel_spread=0.2, divergence=2e-3, x_mean=-2.0, x_sigma=1.0,
                   r_sigma=1.0, id0=0)
    spec = {"kind": W.FIELD_PW, "circular": 0, "a0": 300.0, "ncycles": 8.0, "phase0": 0.3, "pol_angle": 0.4,
            "phi_start": 0.0}
    cfg = {"dt": W.TWO_PI / 500, "procs": procs, "seed": 9, "next_id": 1 << 41}
    return st, spec, cfg, 600, steps


@pytest.mark.parametrize("mode", ["fused", "split"])
def test_photon_vb_nbw_fp64(mode):
    _say(f"photons VB+NBW {mode}")
    st, spec, cfg, s0, steps = _photon_case()
    n = len(st["x"])
    f = oracle.make_field(spec)
    G = oracle.PhotonArrays.from_state(st)
    em, ep = oracle.LeptonArrays.empty(n, -1), oracle.LeptonArrays.empty(n, 1)
    sim = _sim(cfg)
    for s in range(s0, s0 + steps):
        sim.photon_step(f, G, em, ep, s)
    ctx = _ctx(cfg)
    Gg = Q.Photons.from_state(st)
    emg, epg = Q.Leptons(n, -1), Q.Leptons(n, 1)
    segs = Q.whole(spec)
    for s in range(s0, s0 + steps):
        if mode == "fused":
            ctx.step_photons(segs, Gg, emg, epg, s)
        else:
            ctx.birefringence(segs, Gg, s)
            ctx.pair(segs, Gg, emg, epg, s)
    assert em.count > 100, em.count
    _close_pho(Gg.to_numpy(), G.view(), what="photons")
    _close_lep(emg.to_numpy(), em.view(), what="electrons")
    _close_lep(epg.to_numpy(), ep.view(), what="positrons")
    assert ctx.next_id() == sim.next_id
    # compaction
    Gc = Q.Photons(n)
    ctx.compact_photons(Gg, Gc)
    sim.compact(G)
    _close_pho(Gc.to_numpy(), G.view(), what="compacted")


def test_cascade_grid_fp64():
    """Electrons, photons and pairs on a 2D Yee grid in one run: NCS + Stokes + VB + NBW."""
    _say("cascade on grid")
    grid = {"nx": 384, "ny": 96, "dx": W.TWO_PI / 40, "dy": W.TWO_PI / 40, "gx0": -4.8 * math.pi,
            "gy0": -1.2 * math.pi}
    pulse = {"a0": 300.0, "ncycles": 4.0, "w0": 3 * W.TWO_PI, "phi_start": -4 * math.pi}
    comps = W.grid_fill(grid, pulse, 0.0)
    spec_o = dict(kind=W.FIELD_GRID2D, grid=comps, **grid)
    spec_g = dict(kind=W.FIELD_GRID2D, grid=[torch.as_tensor(c).cuda() for c in comps], **grid)
    n = 600
    st = W.beam(n, seed=31, gamma0=4000.0, gamma_rel_spread=0.05, divergence=1e-3, x_mean=0.0,
                x_sigma=0.5, r_sigma=1.0, spin="iso")     # at the peak of the (static) pulse
    cfg = {"dt": W.TWO_PI / 500, "procs": 15, "seed": 3, "next_id": 1 << 40}
    cap = 20 * n
    f = oracle.make_field(spec_o)
    em = oracle.LeptonArrays.from_state(st, capacity=cap, charge=-1)
    ep = oracle.LeptonArrays.empty(cap, 1)
    G = oracle.PhotonArrays.empty(cap)
    sim = _sim(cfg)
    ctx = _ctx(cfg)
    emg = Q.Leptons.from_state(st, capacity=cap, charge=-1)
    epg = Q.Leptons(cap, 1)
    Gg = Q.Photons(cap)
    segs = Q.whole(spec_g)
    for s in range(0, 200):
        sim.step(f, em, ep, G, s)
        ctx.step(segs, emg, epg, Gg, s)
    assert G.count > 500 and ep.count > 0, (G.count, ep.count)
    _close_lep(emg.to_numpy(), em.view(), what="electrons")
    _close_lep(epg.to_numpy(), ep.view(), what="positrons")
    _close_pho(Gg.to_numpy(), G.view(), what="photons")
    assert ctx.next_id() == sim.next_id


# ----------------------------------------------------------------------------- mixed precision
def test_mixed_precision_tracks_fp64():
    """QED_MIXED (FP32 rates, sampling, spin, Stokes, field transcendentals after an FP64
    phase reduction) against the FP64 GPU path on the same inputs and draws: per particle
    within single-precision error, event counts within a handful."""
    _say("mixed vs fp64")
    cfg = W.c2(20000, start_step=2400)
    res = {}
    for prec in (Q.QED_FP64, Q.QED_MIXED):
        ctx = _ctx(cfg, precision=prec)
        Lg = Q.Leptons.from_state(cfg["leptons"], precision=prec)
        Gg = Q.Photons(100000, precision=prec)
        segs = Q.whole(cfg["field"])
        for s in range(2400, 2600):
            ctx.step_leptons(segs, Lg, Gg, s)
        res[prec] = (Lg.to_numpy(), Gg.to_numpy())
    a, b = res[Q.QED_FP64][0], res[Q.QED_MIXED][0]
    ga, gb = res[Q.QED_FP64][1], res[Q.QED_MIXED][1]
    assert len(ga["x"]) > 2000
    assert abs(len(ga["x"]) - len(gb["x"])) <= 5
    e_a = np.sqrt(1 + a["px"] ** 2 + a["py"] ** 2 + a["pz"] ** 2)
    e_b = np.sqrt(1 + b["px"] ** 2 + b["py"] ** 2 + b["pz"] ** 2)
    rel = np.abs(e_b / e_a - 1)
    assert np.median(rel) < 1e-5 and np.mean(rel < 1e-3) > 0.99
    assert abs(e_b.mean() / e_a.mean() - 1) < 1e-3
    Sa = np.stack([a["sx"], a["sy"], a["sz"]])
    Sb = np.stack([b["sx"], b["sy"], b["sz"]])
    assert np.linalg.norm(Sa.mean(axis=1) - Sb.mean(axis=1)) < 2e-3
    assert abs(ga["xi3"].mean() - gb["xi3"].mean()) < 2e-2


@pytest.mark.parametrize("kind", ["pw_lp", "pw_cp", "gauss_cp"])
def test_gathered_fields_both_precisions(kind):
    """qed_gather against the oracle's field evaluation at the bunch positions inside the
    pulse: FP64 to rounding, mixed (FP32 pulse after an FP64 phase reduction, hardware
    sine / cosine / exp) within single-precision error of the amplitude."""
    _say(f"gather {kind}")
    specs = {
        "pw_lp": {"kind": W.FIELD_PW, "circular": 0, "a0": 50.0, "ncycles": 10.0, "phase0": 0.3, "pol_angle": 0.4,
                  "phi_start": 0.0},
        "pw_cp": {"kind": W.FIELD_PW, "circular": 1, "a0": 50.0, "ncycles": 10.0, "phase0": -1.1, "pol_angle": 0.0,
                  "phi_start": 0.0},
        "gauss_cp": W.c2(10, start_step=0)["field"],
    }
    spec = specs[kind]
    cfg = W.c2(3000, start_step=2500)
    st = cfg["leptons"]
    step = 2500
    t = step * cfg["dt"]
    want = np.zeros((3000, 6))
    for j in range(3000):
        E, B = oracle.field_eval(spec, t, [st["x"][j], st["y"][j], st["z"][j]])
        want[j, :3], want[j, 3:] = E, B
    a0 = spec["a0"]
    assert np.max(np.abs(want)) > 0.3 * a0   # the bunch sits inside the pulse
    for prec, tol in ((Q.QED_FP64, 1e-12), (Q.QED_MIXED, 4e-6)):
        ctx = _ctx(cfg, precision=prec)
        Lg = Q.Leptons.from_state(st, precision=prec)
        E6 = torch.zeros(3000 * 6, dtype=torch.float64, device="cuda")
        ctx.gather(Q.whole(spec), Lg, E6, step)
        got = E6.view(3000, 6).cpu().numpy()
        err = np.max(np.abs(got - want)) / a0
        assert err < tol, (prec, err)


@pytest.mark.parametrize("nx,ny", [(3, 1), (7, 5), (40, 24)])
def test_grid_gather_edges(nx, ny):
    """TSC gather from a 2D grid of random values at positions inside, on the border of and
    beyond the grid in both directions (taps partly or wholly off the grid), for the
    narrowest grid the kernels accept and ragged ones: FP64 to rounding, mixed within
    single-precision error."""
    _say(f"grid gather edges {nx}x{ny}")
    rng = np.random.default_rng(7 + nx)
    dx, dy, gx0, gy0 = 0.7, 0.45, -1.3, 2.1
    comps = [rng.uniform(-1.0, 1.0, (ny, nx)).astype(np.float32) for _ in range(6)]
    spec_o = dict(kind=W.FIELD_GRID2D, grid=comps, nx=nx, ny=ny, dx=dx, dy=dy, gx0=gx0, gy0=gy0)
    spec_g = dict(spec_o, grid=[torch.as_tensor(c).cuda() for c in comps])
    n = 1500
    st = W.beam(n, seed=70 + nx, gamma0=10.0, gamma_rel_spread=0.1, divergence=1e-2, x_mean=0.0, x_sigma=1.0,
                r_sigma=1.0)
    st["x"] = gx0 + dx * rng.uniform(-3.0, nx + 2.0, n)
    st["y"] = gy0 + dy * rng.uniform(-3.0, ny + 2.0, n)
    want = np.zeros((n, 6))
    for j in range(n):
        E, B = oracle.field_eval(spec_o, 0.0, [st["x"][j], st["y"][j], st["z"][j]])
        want[j, :3], want[j, 3:] = E, B
    off = np.all(want == 0.0, axis=1)
    assert off.any() and np.sum(~off) > 300    # both wholly-off and on-grid positions
    cfg = W.c1(10)
    for prec, tol in ((Q.QED_FP64, 1e-12), (Q.QED_MIXED, 2e-6)):
        ctx = _ctx(cfg, precision=prec)
        Lg = Q.Leptons.from_state(st, precision=prec)
        E6 = torch.zeros(n * 6, dtype=torch.float64, device="cuda")
        ctx.gather(Q.whole(spec_g), Lg, E6, 0)
        got = E6.view(n, 6).cpu().numpy()
        err = np.max(np.abs(got - want))
        assert err < tol, (prec, err)
    with pytest.raises(RuntimeError):
        narrow = dict(spec_g, nx=2, grid=[c[:, :2].contiguous() for c in spec_g["grid"]])
        ctx.gather(Q.whole(narrow), Lg, E6, 0)


def test_step_events_bracket_the_launches():
    """qed_set_step_events: the four events bracket decide, scan and event kernel in order,
    and switching them off leaves the results unchanged (bitwise)."""
    _say("step events")
    cfg = W.c2(5000, start_step=2450)
    out = []
    for timed in (False, True):
        ctx = _ctx(cfg, precision=Q.QED_MIXED)
        Lg = Q.Leptons.from_state(cfg["leptons"], precision=Q.QED_MIXED)
        Gg = Q.Photons(20000, precision=Q.QED_MIXED)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for s in range(2450, 2460):
            if timed:
                ctx.set_step_events(ev)
            ctx.step_leptons(Q.whole(cfg["field"]), Lg, Gg, s)
        torch.cuda.synchronize()
        if timed:
            ctx.set_step_events(None)
            parts = [ev[k].elapsed_time(ev[k + 1]) for k in range(3)]
            assert all(x >= 0 for x in parts)
            assert abs(sum(parts) - ev[0].elapsed_time(ev[3])) < 1e-3 + 1e-6 * sum(parts)
        out.append((Lg.to_numpy(), Gg.to_numpy()))
    for k in out[0][0]:
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    for k in out[0][1]:
        assert np.array_equal(out[0][1][k], out[1][1][k]), k


# ----------------------------------------------------------------------------- full size
def _sampled_full_size(precision):
    cfg = W.c2(10_000_000, start_step=2500)
    n = 10_000_000
    step = 2500
    ctx = _ctx(cfg, precision=precision)
    Lg = Q.Leptons.from_state(cfg["leptons"], precision=precision)
    Gg = Q.Photons(2_000_000, precision=precision)
    ctx.step_leptons(Q.whole(cfg["field"]), Lg, Gg, step)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(n, 3000, replace=False))
    sample = {k: v[idx].copy() for k, v in cfg["leptons"].items()}
    L = oracle.LeptonArrays.from_state(sample)
    G = oracle.PhotonArrays.empty(3000)
    sim = _sim(cfg)
    sim.step(oracle.make_field(cfg["field"]), L, None, G, step)
    ti = torch.as_tensor(idx).cuda()
    g = {k: getattr(Lg, k)[ti].double().cpu().numpy() for k in Q.LEPTON_KEYS}
    g["id"] = Lg.id[ti].cpu().numpy().view(np.uint64)
    return g, L.view(), Gg.to_numpy(), G.view(), ctx, cfg


def test_full_size_c2_step_sampled_fp64():
    """One fused step of the 1e7-electron focused-pulse workload (the benchmark's launch
    configuration): sampled particles against the oracle, emitted photons found by their
    birth position and checked one by one; the photon list is ordered by parent index."""
    _say("full size c2 fp64 sampled")
    g, o, gp, op, ctx, cfg = _sampled_full_size(Q.QED_FP64)
    _close_lep(g, o, what="sampled leptons")
    assert len(gp["x"]) > 10000
    ids = gp["id"]
    assert np.array_equal(ids, cfg["next_id"] + np.arange(len(ids), dtype=np.uint64))
    gx = np.stack([gp["x"], gp["y"], gp["z"]])
    for j in range(len(op["x"])):
        d = np.sum((gx - np.array([op["x"][j], op["y"][j], op["z"][j]])[:, None]) ** 2, axis=0)
        h = int(np.argmin(d))
        scale = 1.0 + abs(op["x"][j]) + abs(op["y"][j]) + abs(op["z"][j])
        assert math.sqrt(d[h]) < 1e-10 * scale
        assert np.partition(d, 1)[1] > 1e-12 * scale ** 2     # the match is unique
        for k in ("kx", "ky", "kz"):
            assert abs(gp[k][h] - op[k][j]) <= 1e-10 * (abs(op[k][j]) + 1)
        for k in ("xi1", "xi2", "xi3", "e1x", "e1y", "e1z"):
            assert abs(gp[k][h] - op[k][j]) < 1e-10


def test_full_size_c2_step_sampled_mixed():
    _say("full size c2 mixed sampled")
    g, o, gp, op, ctx, cfg = _sampled_full_size(Q.QED_MIXED)
    pm = np.sqrt(o["px"] ** 2 + o["py"] ** 2 + o["pz"] ** 2)
    for k in ("px", "py", "pz"):
        assert np.median(np.abs(g[k] - o[k]) / pm) < 1e-6
    dS = np.sqrt((g["sx"] - o["sx"]) ** 2 + (g["sy"] - o["sy"]) ** 2 + (g["sz"] - o["sz"]) ** 2)
    assert np.mean(dS < 1e-4) > 0.99


def test_multi_segment_collisions_fp64():
    """Several collisions in one list (one segment each: different lasers, one launch):
    equal to running every collision separately in index order with one photon list."""
    _say("multi-segment")
    specs = [
        {"kind": W.FIELD_PW, "circular": 0, "a0": 20.0, "ncycles": 8.0, "phase0": 0.0, "pol_angle": 0.0,
         "phi_start": 0.0},
        {"kind": W.FIELD_PW, "circular": 1, "a0": 35.0, "ncycles": 6.0, "phase0": 0.5, "pol_angle": 0.3,
         "phi_start": 2.0},
        {"kind": W.FIELD_GAUSS, "circular": 1, "a0": 60.0, "ncycles": 8.0, "phase0": 0.0, "pol_angle": 0.0,
         "w0": 3 * W.TWO_PI, "x_focus": 0.0, "phi_start": 0.0},
    ]
    sizes = [700, 1300, 257]
    states = [W.beam(m, seed=70 + k, gamma0=1500.0, gamma_rel_spread=0.05, divergence=1e-3, x_mean=8.0,
                     x_sigma=1.0, r_sigma=2.0, spin="iso", id0=sum(sizes[:k])) for k, m in enumerate(sizes)]
    cfg = {"dt": W.TWO_PI / 400, "procs": oracle.PROC_NCS | oracle.PROC_NCS_STOKES, "seed": 4, "next_id": 1 << 40}
    # oracle: collisions one after the other, shared photon list and id counter
    sim = _sim(cfg)
    G = oracle.PhotonArrays.empty(40000)
    Ls = [oracle.LeptonArrays.from_state(st) for st in states]
    fs = [oracle.make_field(sp) for sp in specs]
    # gpu: one list, three segments
    full = {k: np.concatenate([st[k] for st in states]) for k in states[0]}
    ctx = _ctx(cfg)
    Lg = Q.Leptons.from_state(full)
    Gg = Q.Photons(40000)
    bounds = np.cumsum([0] + sizes)
    segs = Q.segments([(bounds[k], bounds[k + 1], specs[k]) for k in range(3)])
    for s in range(0, 120):
        for L, f in zip(Ls, fs):
            sim.step(f, L, None, G, s)
        ctx.step_leptons(segs, Lg, Gg, s)
    assert G.count > 500
    ov = {k: np.concatenate([L.view()[k] for L in Ls]) for k in Ls[0].view()}
    _close_lep(Lg.to_numpy(), ov, what="leptons")
    _close_pho(Gg.to_numpy(), G.view(), what="photons")
    assert ctx.next_id() == sim.next_id

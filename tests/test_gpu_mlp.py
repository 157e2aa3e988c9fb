"""GPU tests of the learned NCS sampler against the oracle: training pairs (inputs and
targets), the BF16 matrix-core forward pass, the FP32 gradient, and training itself."""
import numpy as np
import pytest

import oracle
import oracle.mlp as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2306_11288_amd as Q  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    Q.lib()


def _say(msg):
    print(f"[gpu-mlp] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_init(seed=11)
    return c


def _denorm(X):
    X = X.astype(np.float64)
    chi = 10.0 ** (2.35 * X[:, 0] - 0.65)
    return chi, X[:, 1], X[:, 2], 0.5 * (X[:, 3] + 1.0)


def test_training_pairs_match_oracle(ctx):
    _say("training pairs")
    X, Y = ctx.mlp_samples(3000, seed=5)
    X, Y = X.cpu().numpy(), Y.cpu().numpy()
    chi, s, c, r = _denorm(X)
    assert chi.min() >= 0.99e-3 and chi.max() <= 50.5 and np.all(s * s + c * c <= 1 + 1e-6)
    assert np.all((r > 0) & (r < 1))
    want = M.normalise_targets(oracle.tables().sampler_targets(chi, s, c, r))
    err = np.abs(Y - want)
    assert err[:, 0].max() < 2e-6, err[:, 0].max()
    assert err[:, 1:].max() < 2e-6, err[:, 1:].max()
    # inputs cover the domain
    assert X[:, 0].min() < -0.95 and X[:, 0].max() > 0.95 and abs(X[:, 3].mean()) < 0.05


@pytest.mark.parametrize("scale", [0.12, 0.2])
def test_forward_matches_oracle(ctx, scale):
    """Random weights large enough for O(1) outputs, a ragged last tile."""
    _say(f"forward {scale}")
    theta = np.random.default_rng(int(scale * 100)).normal(0.0, scale, Q.MLP_NPARAM).astype(np.float32)
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_set_params(theta)
    theta = c.mlp_get_params().cpu().numpy().astype(np.float64)
    X, _ = ctx.mlp_samples(4096 + 37, seed=6)
    ctx = c
    Y = ctx.mlp_forward(X).cpu().numpy()
    Xn = X.cpu().numpy()
    emu = M.forward_bf16(theta, Xn)
    exact, _ = M.forward(theta, Xn)
    assert np.std(exact) > 0.1   # the outputs are not trivially small
    assert np.max(np.abs(Y - emu)) < 5e-3 * (1 + np.max(np.abs(emu))), np.max(np.abs(Y - emu))
    assert np.max(np.abs(Y - exact)) < 3e-2 * (1 + np.max(np.abs(exact))), np.max(np.abs(Y - exact))


def test_gradient_matches_oracle(ctx):
    _say("gradient")
    theta = ctx.mlp_get_params().cpu().numpy().astype(np.float64)
    X, T = ctx.mlp_samples(1000, seed=7)
    w = (1.0, 0.3, 0.3)
    loss, g = ctx.mlp_gradient(X, T, w)
    lo, go = M.loss_and_grad(theta, X.cpu().numpy(), T.cpu().numpy(), w)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - lo) < 1e-5 * lo
    assert np.linalg.norm(g - go) < 2e-5 * np.linalg.norm(go), np.linalg.norm(g - go) / np.linalg.norm(go)
    assert np.max(np.abs(g - go)) < 1e-4 * np.max(np.abs(go))


def test_gradient_over_many_slices_ragged(ctx):
    """A batch spread over every slice of the weight-gradient sums (several staged chunks
    each) with a padded tail: the gradient and the loss still match the FP64 backprop."""
    _say("gradient, 20000 samples")
    theta = ctx.mlp_get_params().cpu().numpy().astype(np.float64)
    X, T = ctx.mlp_samples(20000, seed=17)
    w = (1.0, 0.3, 0.3)
    loss, g = ctx.mlp_gradient(X, T, w)
    lo, go = M.loss_and_grad(theta, X.cpu().numpy(), T.cpu().numpy(), w)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - lo) < 1e-5 * lo
    assert np.linalg.norm(g - go) < 2e-5 * np.linalg.norm(go), np.linalg.norm(g - go) / np.linalg.norm(go)


def test_train_step_is_adam_on_the_gradient():
    """One training step is Adam's first step on the batch gradient, and the weight copies
    the kernels read afterwards (FP32 for the backward pass, bf16 for inference) follow."""
    _say("train step")
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_init(seed=21)
    th0 = c.mlp_get_params().cpu().numpy().astype(np.float64)
    X, T = c.mlp_samples(3000, seed=22)
    Xn, Tn = X.cpu().numpy(), T.cpu().numpy()
    w, lr = (1.0, 0.3, 0.3), 1e-3
    _, go = M.loss_and_grad(th0, Xn, Tn, w)
    c.mlp_train_step(X, T, lr=lr, w=w)
    th1 = c.mlp_get_params().cpu().numpy().astype(np.float64)
    # first Adam step: the bias-corrected moments are g and g^2
    want = th0 - lr * go / (np.abs(go) + 1e-8)
    # where the FP32 gradient's sign is certain (its error is below 1e-4 of the largest
    # component) the step is the FP64 one; everywhere its size is at most lr
    big = np.abs(go) > 1e-3 * np.max(np.abs(go))
    assert big.sum() > 1000
    assert np.max(np.abs(th1 - want)[big]) < 2e-3 * lr
    assert np.max(np.abs(th1 - th0)) < lr * (1 + 1e-3)
    # the FP32 transposed copies: the next gradient is the gradient at the new parameters
    X2, T2 = c.mlp_samples(2000, seed=23)
    _, g2 = c.mlp_gradient(X2, T2, w)
    _, g2o = M.loss_and_grad(th1, X2.cpu().numpy(), T2.cpu().numpy(), w)
    g2 = g2.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g2 - g2o) < 2e-5 * np.linalg.norm(g2o)
    # the bf16 copies: inference with the new parameters
    Y = c.mlp_forward(X2).cpu().numpy()
    emu = M.forward_bf16(th1, X2.cpu().numpy())
    assert np.max(np.abs(Y - emu)) < 5e-3 * (1 + np.max(np.abs(emu)))


def test_training_reduces_the_error(ctx):
    _say("training")
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_init(seed=12)
    X, T = c.mlp_samples(1 << 17, seed=8)
    Xv, Tv = c.mlp_samples(1 << 14, seed=9)
    err0 = (c.mlp_forward(Xv) - Tv).abs().mean(0).cpu().numpy()
    B = 2048
    for it in range(600):
        k = (it * B) % (X.shape[0] - B)
        c.mlp_train_step(X[k:k + B], T[k:k + B], lr=2e-3, w=(1.0, 0.3, 0.3))
    err1 = (c.mlp_forward(Xv) - Tv).abs().mean(0).cpu().numpy()
    _say(f"mean abs error before {err0}, after {err1}")
    assert np.all(err1 < 0.25 * err0)
    assert err1[0] < 0.02


@pytest.fixture(scope="module")
def trained():
    """The network shipped with the package (trained on 5e7 pairs by the library)."""
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_load_pretrained()
    return c.mlp_get_params(), None


def test_trained_network_against_table_sampler(trained):
    """The table sampler (FP32 tables of a mixed context) as the reference for the network on fresh
    inputs; the network's weights are 60x smaller than the FP32 spectrum tables."""
    params, res = trained
    c = Q.Context(dt=0.01, procs=Q.PROC_NCS | Q.PROC_NCS_STOKES, seed=1, id_start=0, precision=Q.QED_MIXED)
    c.mlp_set_params(params)
    X, T64 = c.mlp_samples(1 << 16, seed=21)
    Yt = c.sampler_table(X)
    Ym = c.mlp_forward(X)
    d_table = (Yt - T64).abs().mean(0).cpu().numpy()     # FP32 tables vs FP64 tables
    d_mlp = (Ym - T64).abs().mean(0).cpu().numpy()
    _say(f"mean abs error: table(FP32) {d_table}, network {d_mlp}")
    assert d_table[0] < 1e-5
    assert d_mlp[0] < 2e-3 and d_mlp[1] < 3e-3 and d_mlp[2] < 3e-3
    net_bytes = Q.MLP_NPARAM * 2                            # bf16 weights on the matrix cores
    table_bytes = 4 * 2 * 512 * 1024                        # FP32 NCS spectrum table (A, B)
    assert table_bytes > 60 * net_bytes


@pytest.mark.parametrize("precision", [Q.QED_MIXED, Q.QED_FP64], ids=["mixed", "fp64"])
def test_learned_sampler_in_the_step(trained, precision):
    """The focused-pulse step with the network as sampler against the same step with the
    table: identical first-step event decisions and ids, photon spectra close."""
    params, _ = trained
    cfg = __import__("workloads").c2(20000, start_step=2450)
    out = {}
    for sampler in (Q.SAMPLER_TABLE, Q.SAMPLER_MLP):
        c = Q.Context(dt=cfg["dt"], procs=cfg["procs"], seed=cfg["seed"], id_start=cfg["next_id"],
                      precision=precision)
        c.mlp_set_params(params)
        c.set_sampler(sampler)
        L = Q.Leptons.from_state(cfg["leptons"], precision=precision)
        G = Q.Photons(200000, precision=precision)
        c.step_leptons(Q.whole(cfg["field"]), L, G, 2450)
        torch.cuda.synchronize()
        first = G.to_numpy()
        for s in range(2451, 2550):
            c.step_leptons(Q.whole(cfg["field"]), L, G, s)
        torch.cuda.synchronize()
        out[sampler] = (first, G.to_numpy(), L.to_numpy())
    ft, fm = out[Q.SAMPLER_TABLE][0], out[Q.SAMPLER_MLP][0]
    assert len(ft["x"]) == len(fm["x"]) > 50 and np.array_equal(ft["id"], fm["id"])
    assert np.array_equal(ft["x"], fm["x"])                  # same emitters, same birth places
    gt, gm = out[Q.SAMPLER_TABLE][1], out[Q.SAMPLER_MLP][1]
    assert len(gt["x"]) > 2000 and abs(len(gm["x"]) / len(gt["x"]) - 1) < 0.02
    et = np.sqrt(gt["kx"] ** 2 + gt["ky"] ** 2 + gt["kz"] ** 2)
    em = np.sqrt(gm["kx"] ** 2 + gm["ky"] ** 2 + gm["kz"] ** 2)
    assert abs(em.mean() / et.mean() - 1) < 0.005
    # Kolmogorov-Smirnov distance of the photon energy distributions
    grid = np.quantile(et, np.linspace(0.01, 0.99, 99))
    ks = np.max(np.abs(np.searchsorted(np.sort(et), grid) / len(et) - np.searchsorted(np.sort(em), grid) / len(em)))
    _say(f"photons {len(gt['x'])} / {len(gm['x'])}, mean energy ratio {em.mean() / et.mean():.4f}, KS {ks:.4f}")
    assert ks < 0.01


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

"""Pins of the learned sampler's reference pieces (CPU): the FP64 network and its
backpropagation against torch's autograd on the CPU and against central differences;
the sampler targets against the spin sum done explicitly and against the classical
limit of the photon polarisation."""
import numpy as np
import pytest

import oracle
import oracle.mlp as M


def _params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.normal(0.0, scale, M.N_PARAMS)


def _batch(seed, n):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, (n, 4))
    Y = g.uniform(-1, 1, (n, 3))
    return X, Y


def test_forward_and_gradient_match_torch_autograd():
    torch = pytest.importorskip("torch")
    theta = _params(1)
    X, Y = _batch(2, 17)
    w = (1.0, 0.3, 0.3)
    out, _ = M.forward(theta, X)
    loss, grad = M.loss_and_grad(theta, X, Y, w)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    k, h = 0, torch.tensor(X, dtype=torch.float64)
    for li, (i, o) in enumerate(M.SIZES):
        W = th[k:k + i * o].reshape(i, o)
        k += i * o
        b = th[k:k + o]
        k += o
        h = h @ W + b
        if li < len(M.SIZES) - 1:
            h = torch.nn.functional.silu(h)
    tl = (torch.tensor(w, dtype=torch.float64) * (h - torch.tensor(Y)) ** 2).sum() / X.shape[0]
    tl.backward()
    assert np.allclose(out, h.detach().numpy(), rtol=1e-13, atol=1e-13)
    assert abs(loss - tl.item()) < 1e-13 * max(1.0, abs(loss))
    assert np.allclose(grad, th.grad.numpy(), rtol=1e-11, atol=1e-13)


def test_gradient_matches_central_differences():
    theta = _params(3)
    X, Y = _batch(4, 9)
    _, grad = M.loss_and_grad(theta, X, Y)
    g = np.random.default_rng(5)
    for k in g.choice(M.N_PARAMS, 40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grad(tp, X, Y)[0] - M.loss_and_grad(tm, X, Y)[0]) / (2 * h)
        assert abs(fd - grad[k]) < 1e-7 * max(1.0, abs(fd)), k


def test_silu_derivative_and_bf16_rounding():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    assert np.allclose(M.silu_prime(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h), atol=1e-9)
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 rounds to 1 (tie to even), 1 + 3*2^-8 up
    assert M.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert M.bf16_round(np.array([-3.0]))[0] == -3.0


@pytest.fixture(scope="module")
def tab():
    return oracle.tables()


def test_targets_equal_explicit_spin_sum(tab):
    """Mean Stokes target = (sum over S_f = +-zeta of F_j) / (sum of F_0) for any zeta,
    with F from the exact Bessel functions (orc_ncs_F)."""
    g = np.random.default_rng(6)
    for _ in range(20):
        chi = 10 ** g.uniform(-3, np.log10(50))
        S = g.normal(size=3)
        S /= np.linalg.norm(S)
        r = g.uniform(0.02, 0.98)
        T = tab.sampler_targets([chi], [S[1]], [S[2]], [r])[0]
        assert abs(T[0] - tab.ncs_sample_t(chi, S[1], r)) == 0.0
        t3 = T[0] ** 3
        u = 1.5 * chi * t3
        zeta = g.normal(size=3)
        zeta /= np.linalg.norm(zeta)
        a, b, n = np.eye(3)
        Fs = np.zeros(4)
        for sgn in (1.0, -1.0):
            Fs += oracle.ncs_F(u, chi, S, sgn * zeta, a, b, n)
        assert abs(T[1] - Fs[3] / Fs[0]) < 1e-6, (chi, T, Fs)
        assert abs(T[2] - Fs[2] / Fs[0]) < 1e-6
        assert abs(T[1]) <= 1 + 1e-12 and abs(T[2]) <= 1 + 1e-12


def test_targets_classical_limit_of_photon_polarisation(tab):
    """Unpolarised electrons (S = 0) at chi -> 0: photons drawn from the spectrum have
    mean linear polarisation xi3 = 3/5 (count weighted) and no circular polarisation."""
    m = 4000
    r = (np.arange(m) + 0.5) / m
    T = tab.sampler_targets(np.full(m, 1e-3), np.zeros(m), np.zeros(m), r)
    assert abs(T[:, 1].mean() - 0.6) < 5e-3
    assert np.max(np.abs(T[:, 2])) == 0.0


def _nbw_explicit_means(chi, xi3, d, zeta):
    """<S+ . b>, <S- . b> at delta = d by summing eqs. (G0)-(G3) (exact Bessel functions,
    orc_nbw_G) over both spins, the partner's along an arbitrary axis zeta."""
    a, b, v = np.eye(3)[0], np.eye(3)[1], np.eye(3)[2]     # b = v x a
    xi = np.array([0.0, 0.0, xi3])

    def W(Sp, Sm):
        G = oracle.nbw_G(d, chi, Sp, Sm, a, b, v)
        return G[0] + xi @ G[1:]
    num_p = num_m = den = 0.0
    for s in (1.0, -1.0):
        for t in (1.0, -1.0):
            wp = W(s * b, t * zeta)          # positron along +-b, electron along +-zeta
            wm = W(t * zeta, s * b)          # electron along +-b, positron along +-zeta
            num_p += s * wp
            num_m += s * wm
            den += wp
    return num_p / den, num_m / den


def test_nbw_targets_equal_explicit_spin_sum(tab):
    """NBW sampler targets: delta is the table sampler's, bit for bit; the mean positron and
    electron spins along b equal the explicit sums of the G functions over both spins."""
    g = np.random.default_rng(11)
    done = 0
    while done < 20:
        chi = 10 ** g.uniform(np.log10(0.2), np.log10(50))
        xi3 = g.uniform(-1, 1)
        r = g.uniform(0.02, 0.98)
        T = tab.nbw_sampler_targets([chi], [xi3], [r])[0]
        assert T[0] == tab.nbw_sample_delta(chi, xi3, r)
        d = T[0]
        if 2 / (3 * chi * d * (1 - d)) > 900:       # beyond the Bessel table
            continue
        zeta = g.normal(size=3)
        zeta /= np.linalg.norm(zeta)
        mp, mm = _nbw_explicit_means(chi, xi3, d, zeta)
        assert abs(T[1] - mp) < 1e-6, (chi, xi3, r, T, mp)
        assert abs(T[2] - mm) < 1e-6, (chi, xi3, r, T, mm)
        done += 1


def test_nbw_targets_charge_conjugation_and_bounds(tab):
    """Draws r and 1 - r give delta and 1 - delta (the spectrum's mirror), and the positron's
    mean spin at one is minus the electron's at the other; every mean spin within [-1, 1]."""
    m = 64
    g = np.random.default_rng(12)
    chi = 10 ** g.uniform(np.log10(0.1), np.log10(50), m)
    xi3 = g.uniform(-1, 1, m)
    r = g.uniform(0.01, 0.49, m)
    A = tab.nbw_sampler_targets(chi, xi3, r)
    B = tab.nbw_sampler_targets(chi, xi3, 1 - r)
    assert np.allclose(A[:, 0] + B[:, 0], 1.0, rtol=0, atol=1e-12)
    assert np.allclose(A[:, 1], -B[:, 2], rtol=0, atol=1e-9)
    assert np.allclose(A[:, 2], -B[:, 1], rtol=0, atol=1e-9)
    assert np.all(np.abs(np.concatenate([A[:, 1:], B[:, 1:]])) <= 1 + 1e-12)
    # a soft positron (delta < 1/2, so xi3 / e_- < 1 / e_+) is polarised against b
    assert np.all(A[:, 1] < 0)

"""Oracle pins of the detector diagnostics (the post-processing step of the VB algorithm,
Sec. III.F: rotate each photon's Stokes vector to the detector's polarisation basis and
average per detector cell):

  * rotation to the photon's own basis is the identity; by 90 degrees it flips xi1 and
    xi3; by 45 degrees it exchanges them (xi1' = xi3, xi3' = -xi1); it keeps |xi| and xi2;
  * binning against a brute-force count with the same definitions (slopes, floor, log10
    edges by comparison), particles heading away from the detector and outside the
    ranges excluded; lepton bins sum the spins.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _one_photon(k, e1, xi, w=1.0):
    st = {"x": np.zeros(1), "y": np.zeros(1), "z": np.zeros(1), "kx": np.array([k[0]]), "ky": np.array([k[1]]),
          "kz": np.array([k[2]]), "w": np.array([w]), "xi1": np.array([xi[0]]), "xi2": np.array([xi[1]]),
          "xi3": np.array([xi[2]]), "e1x": np.array([e1[0]]), "e1y": np.array([e1[1]]), "e1z": np.array([e1[2]]),
          "id": np.zeros(1, np.uint64), "alive": np.ones(1, np.uint8)}
    return oracle.PhotonArrays.from_state(st)


def _rotated(k, e1, xi, pol_ref):
    h = oracle.hist_spec((oracle.AX_SLOPE_Y, oracle.AX_SLOPE_Z), (1, 1), (-1, -1), (1, 1), pol_ref)
    out = oracle.hist_photons(_one_photon(k, e1, xi), 0, h)[0, 0]
    assert out[0] == 1.0 and out[1] == pytest.approx(np.linalg.norm(k), rel=1e-15)
    return out[2:]


def test_stokes_rotation_closed_forms():
    xi = np.array([0.3, -0.4, 0.5])
    k = (2e3, 0.0, 0.0)
    assert np.allclose(_rotated(k, (0, 1, 0), xi, (0, 1, 0)), xi, atol=1e-15)          # own basis
    assert np.allclose(_rotated(k, (0, 0, 1), xi, (0, 1, 0)), [-xi[0], xi[1], -xi[2]], atol=1e-15)   # 90 deg
    r = 1 / math.sqrt(2)
    assert np.allclose(_rotated(k, (0, r, r), xi, (0, 1, 0)), [xi[2], xi[1], -xi[0]], atol=1e-15)    # 45 deg


def test_stokes_rotation_keeps_the_degree_and_xi2():
    rng = np.random.default_rng(3)
    for _ in range(50):
        k = np.array([1.0, *rng.normal(0, 0.05, 2)]) * 1e3
        e1 = rng.normal(size=3)
        e1 -= k * (e1 @ k) / (k @ k)
        e1 /= np.linalg.norm(e1)
        xi = rng.normal(size=3)
        xi *= rng.uniform(0, 1) / np.linalg.norm(xi)
        ref = rng.normal(size=3)
        out = _rotated(k, e1, xi, ref)
        assert np.linalg.norm(out) == pytest.approx(np.linalg.norm(xi), rel=1e-13, abs=1e-15)
        assert out[1] == xi[1]


def _brute_bin(v, axis, n, lo, hi):
    if axis == oracle.AX_ENERGY:
        w = (hi - lo) / n
        edges = [math.pow(10.0, lo + i * w) for i in range(n + 1)]
        if not (edges[0] <= v < edges[n]):
            return -1
        return max(i for i in range(n) if edges[i] <= v)
    x = math.floor((v - lo) * (n / (hi - lo)))
    return int(x) if 0 <= x < n else -1


def test_photon_binning_against_brute_force():
    rng = np.random.default_rng(4)
    n = 3000
    st = W.photons(n, seed=5, eps0=300.0, eps_rel_spread=0.6, divergence=0.02, x_mean=0, x_sigma=1, r_sigma=1, id0=0)
    st["kx"][:50] *= -1                        # heading away from the detector
    st["alive"][50:80] = 0                     # removed by a pair event
    st["w"] = rng.uniform(0.5, 2.0, n)
    G = oracle.PhotonArrays.from_state(st)
    axes, nb, lo, hi = (oracle.AX_SLOPE_Y, oracle.AX_ENERGY), (16, 12), (-0.03, 1.0), (0.03, 3.2)
    h = oracle.hist_spec(axes, nb, lo, hi, (0, 0, 1))
    got = oracle.hist_photons(G, 100, h)      # binned from index 100 on
    want = np.zeros((nb[1], nb[0]))
    wsum = np.zeros((nb[1], nb[0]))
    for j in range(100, n):
        kx, ky, kz = st["kx"][j], st["ky"][j], st["kz"][j]
        if not st["alive"][j] or not kx > 0:
            continue
        eps = math.sqrt(kx * kx + ky * ky + kz * kz)
        a = _brute_bin(ky / kx, axes[0], nb[0], lo[0], hi[0])
        b = _brute_bin(eps, axes[1], nb[1], lo[1], hi[1])
        if a >= 0 and b >= 0:
            want[b, a] += 1
            wsum[b, a] += st["w"][j] * eps
    assert got[..., 1] == pytest.approx(wsum, rel=1e-13)
    assert 100 < want.sum() < n - 100 and np.count_nonzero(want) > 20
    st2 = dict(st, w=np.ones(n))
    got2 = oracle.hist_photons(oracle.PhotonArrays.from_state(st2), 100, h)
    assert np.array_equal(got2[..., 0], want)   # counts exact


def test_lepton_binning_sums_the_spins():
    cfg = W.c2(2000)
    st = cfg["leptons"]
    L = oracle.LeptonArrays.from_state(st)
    h = oracle.hist_spec((oracle.AX_SLOPE_R, oracle.AX_ENERGY), (5, 4), (0.0, 3.0), (4e-3, 3.6))
    got = oracle.hist_leptons(L, 0, h)
    p = np.stack([st["px"], st["py"], st["pz"]])
    g = np.sqrt(1 + (p * p).sum(0))
    tot = np.zeros((4, 5, 5))
    for i in range(2000):
        a = _brute_bin(math.sqrt(p[1, i] ** 2 + p[2, i] ** 2) / p[0, i], oracle.AX_SLOPE_R, 5, 0.0, 4e-3)
        b = _brute_bin(g[i], oracle.AX_ENERGY, 4, 3.0, 3.6)
        if a >= 0 and b >= 0:
            tot[b, a] += [1, g[i], st["sx"][i], st["sy"][i], st["sz"][i]]
    assert np.array_equal(got[..., 0], tot[..., 0])
    assert np.allclose(got, tot, rtol=1e-13, atol=1e-12)
    assert tot[..., 0].sum() > 1000

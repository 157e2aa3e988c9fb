"""When particles born in a step are first stepped: the order of the Spin-QED chain (Sec. IV:
Lorentz push and T-BMT, radiative correction, vacuum birefringence, NBW, NCS).

The push runs before NBW, so a pair created in step n is not pushed in step n; NBW runs
before NCS and NCS only sees the leptons that were pushed, so the pair is not tested for
emission either; NCS runs after VB and NBW, so a photon emitted in step n keeps its birth
state until step n + 1.  The ids follow the chain too: pair ids before photon ids.

The setup makes every test certain: a uniform magnetic field strong enough that the
per-step probabilities of NBW (for the photon) and NCS (for every lepton) exceed one.
"""
import math

import numpy as np

import oracle
from oracle import XI_L

B0 = 206.0          # chi = xi_L |p| B0 ~ 5 at 1e4 m c
DT = 20.0           # per-step probabilities of NBW and NCS well above one here


def _field():
    return oracle.make_field({"kind": oracle.FIELD_CONST, "b0": (0.0, 0.0, B0)})


def _setup():
    g = 1.0e4
    pm = math.sqrt(g * g - 1)
    em = oracle.LeptonArrays.from_state(
        {"x": [0.0], "y": [0.0], "z": [0.0], "px": [pm], "py": [0.0], "pz": [0.0], "w": [1.0],
         "sx": [0.0], "sy": [0.0], "sz": [1.0], "id": np.array([0], np.uint64)}, capacity=8, charge=-1)
    ep = oracle.LeptonArrays.empty(8, charge=1)
    G = oracle.PhotonArrays.from_state(
        {"x": [5.0], "y": [0.0], "z": [0.0], "kx": [1.0e4], "ky": [0.0], "kz": [0.0], "w": [1.0],
         "xi1": [0.0], "xi2": [0.0], "xi3": [1.0], "e1x": [0.0], "e1y": [1.0], "e1z": [0.0],
         "id": np.array([1], np.uint64)}, capacity=16)
    sim = oracle.Sim(dt=DT, procs=oracle.PROC_NCS | oracle.PROC_NCS_STOKES | oracle.PROC_NBW | oracle.PROC_VB,
                     seed=9, next_id=100, p_max=1e9)
    return sim, em, ep, G


def test_probabilities_of_the_setup_exceed_one():
    g = 1.0e4
    chi_e = XI_L * math.sqrt(g * g - 1) * B0
    C = oracle.ALPHA / (math.sqrt(3) * math.pi * XI_L * g)
    assert C * (oracle.ncs_Ia(chi_e) - oracle.ncs_Ib(chi_e)) * DT > 2
    chi_g = XI_L * 1.0e4 * B0
    assert oracle.ALPHA / (math.sqrt(3) * math.pi * XI_L * 1.0e4) * (oracle.nbw_Ja(chi_g) - oracle.nbw_Jb(chi_g)) * DT > 2


def test_newborn_pairs_start_in_the_next_step():
    sim, em, ep, G = _setup()
    n = 7
    sim.step(_field(), em, ep, G, n)
    # NBW converted the photon; the pair sits at the photon's position with momenta along
    # its direction: it was neither pushed (no rotation about B, no move) ...
    assert G.alive[0] == 0
    assert em.count == 2 and ep.count == 1
    for L, i in ((em, 1), (ep, 0)):
        assert (L.x[i], L.y[i], L.z[i]) == (5.0, 0.0, 0.0)
        assert L.py[i] == 0.0 and L.pz[i] == 0.0 and L.px[i] > 0
    # ... nor tested for NCS: the only new photon is the one of the electron that was
    # pushed in this step, born at its x^{n+1}
    assert G.count == 2
    assert (G.x[1], G.y[1], G.z[1]) == (em.x[0], em.y[0], em.z[0])
    # ids: the pair (electron, positron) before the NCS photon, as NBW precedes NCS
    assert (int(em.id[1]), int(ep.id[0]), int(G.id[1])) == (100, 101, 102)
    x_born = np.array([em.x[1], ep.x[0]])
    # step n + 1: the pair is pushed and emits
    sim.step(_field(), em, ep, G, n + 1)
    assert em.x[1] != x_born[0] and ep.x[0] != x_born[1]
    assert em.py[1] != 0.0 and ep.py[0] != 0.0
    born = [(G.x[j], G.y[j], G.z[j]) for j in range(2, G.count) if G.alive[j]]
    assert (em.x[1], em.y[1], em.z[1]) in born and (ep.x[0], ep.y[0], ep.z[0]) in born


def test_ncs_photons_keep_their_birth_state_until_the_next_step():
    """The photon emitted in step n keeps the basis of the emitting electron's frame
    (e1 = a, the electron's acceleration q v x B = -n x B) and its birth position; the
    birefringence frame (E_red = n x B) would have turned its basis to -a and moved it."""
    sim, em, ep, G = _setup()
    sim.step(_field(), em, ep, G, 3)
    k = np.array([G.kx[1], G.ky[1], G.kz[1]])
    nxb = np.cross(k / np.linalg.norm(k), np.array([0.0, 0.0, 1.0]))
    nxb /= np.linalg.norm(nxb)
    assert np.array([G.e1x[1], G.e1y[1], G.e1z[1]]) @ (-nxb) > 1 - 1e-12
    assert G.alive[1] == 1
    x1 = np.array([G.x[1], G.y[1], G.z[1]])
    sim.step(_field(), em, ep, G, 4)
    if G.alive[1]:
        assert not np.array_equal(np.array([G.x[1], G.y[1], G.z[1]]), x1)
        assert np.array([G.e1x[1], G.e1y[1], G.e1z[1]]) @ nxb > 1 - 1e-12

"""Oracle: plain, slow, FP64 CPU reference of the spin/polarisation-resolved SF-QED
particle step (Wan et al., arXiv:2306.11288).

TEST INFRASTRUCTURE ONLY -- imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; never by the product package.  The C source
(``qed_oracle.c``) shares no code with the HIP library.

This module is argument marshalling (ctypes + numpy) around that C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qed_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# another build of the same source (e.g. instrumented by sanitizers) can stand in for it
_LIB_OVERRIDE = os.environ.get("QED_ORACLE_LIB")

PROC_NCS, PROC_NCS_STOKES, PROC_NBW, PROC_VB = 1, 2, 4, 8
ST_OVERFLOW, ST_NAN, ST_PMAX, ST_EPS_LT1, ST_CLAMP = 1, 2, 4, 8, 16
FIELD_NONE, FIELD_CONST, FIELD_PW, FIELD_GAUSS, FIELD_GRID2D = 0, 1, 2, 3, 4
TAB_BESSEL, TAB_NCS_RATE, TAB_NCS_CDF, TAB_NBW_RATE, TAB_NBW_CDF, TAB_VB, TAB_RAD = range(7)
RR_LL, RR_MLL, RR_RBMT = 1, 2, 4

ALPHA = 1.0 / 137.035999084          # CODATA 2018
XI_L = 2.42631023867e-6              # hbar omega / m c^2 at lambda = 1 um (= lambda_C/lambda)
A_E = 1.15965218128e-3               # electron anomalous magnetic moment (CODATA 2018)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        d, i64, u32, u64, vp = C.c_double, C.c_int64, C.c_uint32, C.c_uint64, C.c_void_p
        dp = C.POINTER(C.c_double)
        sig = {
            "orc_philox4x32_10": (None, [vp, vp, vp]),
            "orc_uniform4": (None, [u64, i64, u32, u64, vp]),
            "orc_bessel_k": (d, [d, d]),
            "orc_int_bessel_k": (d, [d, d]),
            "orc_scorer_gi_prime": (d, [d]),
            "orc_ncs_Ia": (d, [d]), "orc_ncs_Ib": (d, [d]),
            "orc_ncs_A": (d, [d, d]), "orc_ncs_B": (d, [d, d]),
            "orc_ncs_power_ratio": (d, [d]),
            "orc_rbmt_psi": (None, [d, vp]),
            "orc_nbw_Ja": (d, [d]), "orc_nbw_Jb": (d, [d]),
            "orc_nbw_Ka": (d, [d, d]), "orc_nbw_Kb": (d, [d, d]),
            "orc_vb_M": (None, [d, vp]),
            "orc_ncs_F": (None, [d, d, vp, vp, vp, vp, vp, vp]),
            "orc_nbw_G": (None, [d, d, vp, vp, vp, vp, vp, vp]),
            "orc_tables_build": (vp, []),
            "orc_tables_free": (None, [vp]),
            "orc_tables_size": (i64, [C.c_int]),
            "orc_tables_export": (None, [vp, C.c_int, vp]),
            "orc_tab_bessel": (None, [vp, d, vp]),
            "orc_tab_ncs_rate": (None, [vp, d, dp, dp]),
            "orc_tab_ncs_sample_t": (d, [vp, d, d, d]),
            "orc_sampler_targets_n": (None, [vp, i64, vp, vp, vp, vp, vp]),
            "orc_tab_nbw_rate": (None, [vp, d, dp, dp]),
            "orc_tab_nbw_sample_delta": (d, [vp, d, d, d]),
            "orc_nbw_sampler_targets_n": (None, [vp, i64, vp, vp, vp, vp]),
            "orc_tab_vb_M": (None, [vp, d, vp]),
            "orc_field_eval": (None, [vp, d, vp, vp, vp]),
            "orc_push_spin": (None, [vp, vp, vp, i64, vp]),
            "orc_push_radiative": (None, [vp, vp, vp, vp, i64, u32]),
            "orc_hist_photons": (None, [vp, i64, vp, vp]),
            "orc_hist_leptons": (None, [vp, i64, vp, vp]),
            "orc_ll_force": (None, [d, d, d, vp, vp, vp, vp]),
            "orc_tab_rad": (None, [vp, d, vp]),
            "orc_emit": (None, [vp, vp, vp, vp, vp, i64]),
            "orc_photon_step": (None, [vp, vp, vp, vp, vp, vp, i64]),
            "orc_compact_photons": (i64, [vp]),
            "orc_boris": (None, [d, d, vp, vp, vp, vp, vp]),
            "orc_bmt": (None, [d, d, d, vp, vp, vp, vp, vp]),
            "orc_chi_e": (d, [d, vp, vp, vp]),
            "orc_chi_gamma": (d, [d, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


# ------------------------------------------------------------------ scalar helpers
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def uniform4(pid: int, step: int, stream: int, seed: int) -> np.ndarray:
    r = np.zeros(4)
    lib().orc_uniform4(pid, step, stream, seed, _p(r))
    return r


def bessel_k(nu, x):
    return lib().orc_bessel_k(float(nu), float(x))


def int_bessel_k(nu, x):
    return lib().orc_int_bessel_k(float(nu), float(x))


def scorer_gi_prime(x):
    return lib().orc_scorer_gi_prime(float(x))


def ncs_Ia(chi):
    return lib().orc_ncs_Ia(float(chi))


def ncs_Ib(chi):
    return lib().orc_ncs_Ib(float(chi))


def ncs_A(chi, y):
    return lib().orc_ncs_A(float(chi), float(y))


def ncs_B(chi, y):
    return lib().orc_ncs_B(float(chi), float(y))


def ncs_power_ratio(chi):
    return lib().orc_ncs_power_ratio(float(chi))


def rbmt_psi(chi) -> np.ndarray:
    o = np.zeros(3)
    lib().orc_rbmt_psi(float(chi), _p(o))
    return o


def nbw_Ja(chi):
    return lib().orc_nbw_Ja(float(chi))


def nbw_Jb(chi):
    return lib().orc_nbw_Jb(float(chi))


def nbw_Ka(chi, d):
    return lib().orc_nbw_Ka(float(chi), float(d))


def nbw_Kb(chi, d):
    return lib().orc_nbw_Kb(float(chi), float(d))


AX_SLOPE_Y, AX_SLOPE_Z, AX_SLOPE_R, AX_ENERGY = 0, 1, 2, 3


class HistSpec(C.Structure):
    _fields_ = [("axis", C.c_int32 * 2), ("n", C.c_int32 * 2), ("lo", C.c_double * 2), ("hi", C.c_double * 2),
                ("pol_ref", C.c_double * 3)]


def hist_spec(axes, n, lo, hi, pol_ref=(0.0, 1.0, 0.0)) -> HistSpec:
    h = HistSpec()
    for k in range(2):
        h.axis[k], h.n[k], h.lo[k], h.hi[k] = int(axes[k]), int(n[k]), float(lo[k]), float(hi[k])
    for k in range(3):
        h.pol_ref[k] = float(pol_ref[k])
    return h


def hist_photons(G, begin: int, h: HistSpec) -> np.ndarray:
    """Detector histogram of photons [begin, count): array [n1][n0][5] of
    (w, w eps, w xi1, w xi2, w xi3) with the Stokes vector in the detector basis."""
    out = np.zeros(h.n[0] * h.n[1] * 5)
    s = G.ctype()
    lib().orc_hist_photons(C.byref(s), int(begin), C.byref(h), _p(out))
    return out.reshape(h.n[1], h.n[0], 5)


def hist_leptons(L, begin: int, h: HistSpec) -> np.ndarray:
    """The same for leptons: (w, w gamma, w Sx, w Sy, w Sz)."""
    out = np.zeros(h.n[0] * h.n[1] * 5)
    s = L.ctype()
    lib().orc_hist_leptons(C.byref(s), int(begin), C.byref(h), _p(out))
    return out.reshape(h.n[1], h.n[0], 5)


def ll_force(g, p, E, B, alpha=None, xi_L=None) -> np.ndarray:
    """Classical Landau-Lifshitz force (two leading terms, Sec. III.A.1) at momentum p
    with Lorentz factor g."""
    F = np.zeros(3)
    lib().orc_ll_force(float(alpha if alpha is not None else ALPHA), float(xi_L if xi_L is not None else XI_L),
                       float(g), _p(_f64(p)), _p(_f64(E)), _p(_f64(B)), _p(F))
    return F


def vb_M(chi) -> np.ndarray:
    o = np.zeros(2)
    lib().orc_vb_M(float(chi), _p(o))
    return o


def ncs_F(u, chi, Si, Sf, a, b, n) -> np.ndarray:
    o = np.zeros(4)
    args = [_f64(v) for v in (Si, Sf, a, b, n)]
    lib().orc_ncs_F(float(u), float(chi), *[_p(v) for v in args], _p(o))
    return o


def nbw_G(delta, chi, Sp, Sm, a, b, v) -> np.ndarray:
    o = np.zeros(4)
    args = [_f64(x) for x in (Sp, Sm, a, b, v)]
    lib().orc_nbw_G(float(delta), float(chi), *[_p(x) for x in args], _p(o))
    return o


def boris(q, dt, E, B, p):
    p = _f64(p).copy()
    pm, pp = np.zeros(3), np.zeros(3)
    lib().orc_boris(float(q), float(dt), _p(_f64(E)), _p(_f64(B)), _p(p), _p(pm), _p(pp))
    return p, pm, pp


def bmt(q, a_e, dt, E, B, pm, pp, S):
    S = _f64(S).copy()
    lib().orc_bmt(float(q), float(a_e), float(dt), _p(_f64(E)), _p(_f64(B)), _p(_f64(pm)),
                  _p(_f64(pp)), _p(S))
    return S


def chi_e(p, E, B, xi_L=XI_L):
    return lib().orc_chi_e(xi_L, _p(_f64(p)), _p(_f64(E)), _p(_f64(B)))


def chi_gamma(k, E, B, xi_L=XI_L):
    return lib().orc_chi_gamma(xi_L, _p(_f64(k)), _p(_f64(E)), _p(_f64(B)))


# ------------------------------------------------------------------ tables
class Tables:
    """The oracle's own build of the table specification."""

    def __init__(self):
        self.h = lib().orc_tables_build()

    def __del__(self):
        try:
            if self.h:
                lib().orc_tables_free(self.h)
        except Exception:
            pass

    def export(self, which: int) -> np.ndarray:
        n = lib().orc_tables_size(which)
        o = np.zeros(n)
        lib().orc_tables_export(self.h, which, _p(o))
        return o

    def bessel(self, x) -> np.ndarray:
        o = np.zeros(3)
        lib().orc_tab_bessel(self.h, float(x), _p(o))
        return o

    def ncs_rate(self, chi):
        a, b = C.c_double(), C.c_double()
        lib().orc_tab_ncs_rate(self.h, float(chi), C.byref(a), C.byref(b))
        return a.value, b.value

    def ncs_sample_t(self, chi, s, r):
        return lib().orc_tab_ncs_sample_t(self.h, float(chi), float(s), float(r))

    def sampler_targets(self, chi, s, c, r) -> np.ndarray:
        """[n, 3]: table-sampler t and spin-summed mean xi3, xi2 (orc_sampler_targets)."""
        chi, s, c, r = (_f64(v) for v in (chi, s, c, r))
        out = np.zeros((len(chi), 3))
        lib().orc_sampler_targets_n(self.h, len(chi), _p(chi), _p(s), _p(c), _p(r), _p(out))
        return out

    def nbw_rate(self, chi):
        a, b = C.c_double(), C.c_double()
        lib().orc_tab_nbw_rate(self.h, float(chi), C.byref(a), C.byref(b))
        return a.value, b.value

    def nbw_sample_delta(self, chi, xi3, r):
        return lib().orc_tab_nbw_sample_delta(self.h, float(chi), float(xi3), float(r))

    def nbw_sampler_targets(self, chi, xi3, r) -> np.ndarray:
        """[n, 3]: table-sampler delta and the mean positron / electron spin along b
        (orc_nbw_sampler_targets)."""
        chi, xi3, r = (_f64(v) for v in (chi, xi3, r))
        out = np.zeros((len(chi), 3))
        lib().orc_nbw_sampler_targets_n(self.h, len(chi), _p(chi), _p(xi3), _p(r), _p(out))
        return out

    def rad(self, chi) -> np.ndarray:
        """g(chi) (emitted / Larmor power) and psi1..psi3 from the RAD table."""
        o = np.zeros(4)
        lib().orc_tab_rad(self.h, float(chi), _p(o))
        return o

    def vb_M(self, chi) -> np.ndarray:
        o = np.zeros(2)
        lib().orc_tab_vb_M(self.h, float(chi), _p(o))
        return o


_tables = None


def tables() -> Tables:
    """Process-wide oracle tables (built once, a few seconds)."""
    global _tables
    if _tables is None:
        _tables = Tables()
    return _tables


# ------------------------------------------------------------------ fields and particles
class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("circular", C.c_int32),
                ("a0", C.c_double), ("ncycles", C.c_double), ("phase0", C.c_double),
                ("pol_angle", C.c_double), ("w0", C.c_double), ("x_focus", C.c_double),
                ("phi_start", C.c_double), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("grid", C.c_void_p * 6), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("gx0", C.c_double), ("gy0", C.c_double)]


class _Leptons(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz", "id")] + \
               [("count", C.c_int64), ("capacity", C.c_int64), ("charge", C.c_int32)]


class _Photons(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "y", "z", "kx", "ky", "kz", "w", "xi1", "xi2", "xi3",
                                          "e1x", "e1y", "e1z", "id", "alive")] + \
               [("count", C.c_int64), ("capacity", C.c_int64)]


class _Config(C.Structure):
    _fields_ = [("xi_L", C.c_double), ("alpha", C.c_double), ("a_e", C.c_double), ("dt", C.c_double),
                ("p_max", C.c_double), ("seed", C.c_uint64), ("next_id", C.c_uint64),
                ("procs", C.c_uint32), ("status", C.c_uint32)]


def make_field(spec: dict):
    """Field descriptor from a plain dict (keys as in workloads.FieldSpec)."""
    f = _Field()
    f.kind = int(spec.get("kind", FIELD_NONE))
    f.circular = int(spec.get("circular", 0))
    for k in ("a0", "ncycles", "phase0", "pol_angle", "w0", "x_focus", "phi_start", "dx", "dy", "gx0", "gy0"):
        setattr(f, k, float(spec.get(k, 0.0)))
    for i, v in enumerate(spec.get("e0", (0, 0, 0))):
        f.e0[i] = float(v)
    for i, v in enumerate(spec.get("b0", (0, 0, 0))):
        f.b0[i] = float(v)
    keep = []
    if f.kind == FIELD_GRID2D:
        grids = spec["grid"]
        f.nx, f.ny = int(spec["nx"]), int(spec["ny"])
        for c in range(6):
            g = np.ascontiguousarray(np.asarray(grids[c], dtype=np.float32))
            keep.append(g)
            f.grid[c] = g.ctypes.data
    f._keep = keep
    return f


def field_eval(spec: dict, t, r):
    f = make_field(spec)
    E, B = np.zeros(3), np.zeros(3)
    lib().orc_field_eval(C.byref(f), float(t), _p(_f64(r)), _p(E), _p(B))
    return E, B


def field_eval_points(spec: dict, t, pts):
    """E, B ([n][3] each) of the field at the points pts ([n][3]) at time t."""
    f = make_field(spec)
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    E, B = np.zeros_like(pts), np.zeros_like(pts)
    ev = lib().orc_field_eval
    for k in range(len(pts)):
        ev(C.byref(f), float(t), _p(pts[k]), _p(E[k]), _p(B[k]))
    return E, B


@dataclass
class LeptonArrays:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    px: np.ndarray
    py: np.ndarray
    pz: np.ndarray
    w: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    sz: np.ndarray
    id: np.ndarray
    count: int
    charge: int

    @classmethod
    def empty(cls, capacity: int, charge: int):
        z = lambda: np.zeros(capacity)
        return cls(z(), z(), z(), z(), z(), z(), z(), z(), z(), z(), np.zeros(capacity, np.uint64), 0, charge)

    @classmethod
    def from_state(cls, st: dict, capacity: int | None = None, charge: int = -1):
        n = len(st["x"])
        cap = capacity or n
        L = cls.empty(cap, charge)
        for k in ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz"):
            getattr(L, k)[:n] = st[k]
        L.id[:n] = st["id"]
        L.count = n
        return L

    def ctype(self):
        s = _Leptons()
        for k in ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz", "id"):
            setattr(s, k, getattr(self, k).ctypes.data)
        s.count, s.capacity, s.charge = self.count, len(self.x), self.charge
        return s

    def view(self) -> dict:
        n = self.count
        return {k: getattr(self, k)[:n].copy() for k in
                ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz", "id")}


@dataclass
class PhotonArrays:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray
    w: np.ndarray
    xi1: np.ndarray
    xi2: np.ndarray
    xi3: np.ndarray
    e1x: np.ndarray
    e1y: np.ndarray
    e1z: np.ndarray
    id: np.ndarray
    alive: np.ndarray
    count: int

    KEYS = ("x", "y", "z", "kx", "ky", "kz", "w", "xi1", "xi2", "xi3", "e1x", "e1y", "e1z")

    @classmethod
    def empty(cls, capacity: int):
        z = lambda: np.zeros(capacity)
        return cls(*[z() for _ in cls.KEYS], np.zeros(capacity, np.uint64), np.zeros(capacity, np.uint8), 0)

    @classmethod
    def from_state(cls, st: dict, capacity: int | None = None):
        n = len(st["x"])
        G = cls.empty(capacity or n)
        for k in cls.KEYS:
            getattr(G, k)[:n] = st[k]
        G.id[:n] = st["id"]
        G.alive[:n] = st.get("alive", np.ones(n, np.uint8))
        G.count = n
        return G

    def ctype(self):
        s = _Photons()
        for k in self.KEYS + ("id", "alive"):
            setattr(s, k, getattr(self, k).ctypes.data)
        s.count, s.capacity = self.count, len(self.x)
        return s

    def view(self) -> dict:
        n = self.count
        return {k: getattr(self, k)[:n].copy() for k in self.KEYS + ("id", "alive")}


def sort_by_bin(arrs, grid: dict, bin_cells: int):
    """The list `arrs` (LeptonArrays or PhotonArrays) reordered by grid bin, as a new list
    of the same capacity: the particles (photons: the live ones) stably sorted by key =
    by nbx + bx, with bx = floor((x - gx0) / (bin_cells dx)) clamped to [0, nbx - 1] (NaN
    to 0), by likewise, nbx = ceil(nx / bin_cells).  This is the plain definition of the
    library's data-layout sort: numpy's stable argsort on that key."""
    n = arrs.count
    nbx = -(-int(grid["nx"]) // bin_cells)
    nby = -(-int(grid["ny"]) // bin_cells)

    def bins(v, v0, d, nb):
        f = np.floor((v - v0) * (1.0 / (bin_cells * d)))
        f = np.where(f >= 0.0, f, 0.0)            # negative and NaN to 0
        return np.minimum(f, nb - 1).astype(np.int64)

    x, y = arrs.x[:n], arrs.y[:n]
    key = bins(y, grid["gy0"], grid["dy"], nby) * nbx + bins(x, grid["gx0"], grid["dx"], nbx)
    sel = np.arange(n)
    if isinstance(arrs, PhotonArrays):
        sel = sel[arrs.alive[:n] != 0]
    order = sel[np.argsort(key[sel], kind="stable")]
    st = {k: v[order] for k, v in arrs.view().items()}
    if isinstance(arrs, PhotonArrays):
        return PhotonArrays.from_state(st, capacity=len(arrs.x))
    return LeptonArrays.from_state(st, capacity=len(arrs.x), charge=arrs.charge)


class Sim:
    """Whole-step driver in the order of the paper's Spin-QED chain (Sec. IV):
    Lorentz push and T-BMT of the electrons, then the positrons alive at the start of the
    step -> vacuum birefringence and NBW of the photons alive at the start of the step
    (frame rotation, VB, pair creation, move) -> NCS of the leptons pushed in this step
    (electrons, then positrons).  Pairs born by NBW in step n are neither pushed nor
    tested for NCS before step n + 1; photons born by NCS in step n see VB and NBW from
    step n + 1 on."""

    def __init__(self, *, dt, procs, seed, next_id, p_max=0.1, xi_L=XI_L, alpha=ALPHA, a_e=A_E,
                 tables_obj: Tables | None = None):
        self.cfg = _Config(xi_L, alpha, a_e, dt, p_max, seed, next_id, procs, 0)
        self.tab = tables_obj if tables_obj is not None else (
            tables() if procs & (PROC_NCS | PROC_NBW | PROC_VB) else None)

    @property
    def status(self) -> int:
        return int(self.cfg.status)

    @property
    def next_id(self) -> int:
        return int(self.cfg.next_id)

    def push_spin(self, field, L: LeptonArrays, step: int, E6: np.ndarray | None = None):
        s = L.ctype()
        lib().orc_push_spin(C.byref(self.cfg), C.byref(field), C.byref(s), step,
                            _p(E6) if E6 is not None else None)

    def push_radiative(self, field, L: LeptonArrays, step: int, mode: int):
        """Lorentz or radiative push (mode: RR_LL or RR_MLL, | RR_RBMT) and spin."""
        s = L.ctype()
        tab = self.tab if self.tab is not None else tables()
        lib().orc_push_radiative(C.byref(self.cfg), tab.h, C.byref(field), C.byref(s), step, mode)

    def emit(self, L: LeptonArrays, E6: np.ndarray, G: PhotonArrays | None, step: int, count: int | None = None):
        """NCS of leptons [0, count) (default: all) with the fields E6 of x^n."""
        s = L.ctype()
        if count is not None:
            s.count = count
        g = G.ctype() if G is not None else None
        lib().orc_emit(C.byref(self.cfg), self.tab.h if self.tab else None, C.byref(s), _p(E6),
                       C.byref(g) if g is not None else None, step)
        if G is not None:
            G.count = int(g.count)

    def photon_step(self, field, G: PhotonArrays, em: LeptonArrays | None, ep: LeptonArrays | None, step: int):
        g = G.ctype()
        sm = em.ctype() if em is not None else None
        sp = ep.ctype() if ep is not None else None
        lib().orc_photon_step(C.byref(self.cfg), self.tab.h if self.tab else None, C.byref(field), C.byref(g),
                              C.byref(sm) if sm is not None else None,
                              C.byref(sp) if sp is not None else None, step)
        if em is not None:
            em.count = int(sm.count)
        if ep is not None:
            ep.count = int(sp.count)

    def compact(self, G: PhotonArrays) -> int:
        g = G.ctype()
        G.count = int(lib().orc_compact_photons(C.byref(g)))
        return G.count

    def step(self, field, em: LeptonArrays | None, ep: LeptonArrays | None, G: PhotonArrays | None, step: int,
             photon_procs: bool | None = None):
        if photon_procs is None:
            photon_procs = bool(self.cfg.procs & (PROC_NBW | PROC_VB))
        pushed = []
        for L in (em, ep):          # Lorentz & T-BMT
            if L is None or L.count == 0:
                continue
            E6 = np.zeros(6 * L.count)
            self.push_spin(field, L, step, E6)
            pushed.append((L, L.count, E6))
        if G is not None and photon_procs:   # VB, NBW (pairs appended after the pushed leptons)
            self.photon_step(field, G, em, ep, step)
        if self.cfg.procs & PROC_NCS:        # NCS of the leptons pushed above
            for L, n0, E6 in pushed:
                self.emit(L, E6, G, step, count=n0)

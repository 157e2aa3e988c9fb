"""Python binding of libqed (the HIP/gfx950 spin/polarisation-resolved SF-QED particle
step).  Argument marshalling only: every step of the path runs in the library's kernels.
PyTorch provides device memory and streams.

The C ABI is declared in include/qed.h; the functions here carry the same names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqed.so")

QED_OK, QED_EARG, QED_ENOMEM, QED_EHIP, QED_ESTATE = range(5)
QED_FP64, QED_MIXED = 0, 1
PROC_NCS, PROC_NCS_STOKES, PROC_NBW, PROC_VB = 1, 2, 4, 8
ST_OVERFLOW, ST_NAN, ST_PMAX, ST_EPS_LT1, ST_CLAMP, ST_SCAN, ST_DEPOSIT = 1, 2, 4, 8, 16, 32, 64
FIELD_NONE, FIELD_CONST, FIELD_PW, FIELD_GAUSS, FIELD_GRID2D = 0, 1, 2, 3, 4
TAB_BESSEL, TAB_NCS_RATE, TAB_NCS_CDF, TAB_NBW_RATE, TAB_NBW_CDF, TAB_VB, TAB_RAD = range(7)
RR_LL, RR_MLL, RR_RBMT = 1, 2, 4
EXPORTED = ["qed_init_tables", "qed_destroy", "qed_gather", "qed_push_spin", "qed_push_radiative", "qed_emit",
            "qed_step_leptons", "qed_step_leptons_noalloc",
            "qed_birefringence", "qed_pair", "qed_step_photons", "qed_step", "qed_compact_photons", "qed_sort_photons", "qed_sort_leptons", "qed_read_status",
            "qed_clear_status", "qed_get_next_id", "qed_set_next_id", "qed_table_size", "qed_table_export",
            "qed_set_step_events", "qed_set_photon_events", "qed_set_step_counter", "qed_advance_step", "qed_get_tuning",
            "qed_set_tuning", "qed_autotune", "qed_mlp_init", "qed_mlp_set_params", "qed_mlp_get_params",
            "qed_mlp_samples", "qed_mlp_forward", "qed_mlp_gradient", "qed_mlp_train_step", "qed_set_sampler", "qed_mlp_select", "qed_set_deposit_path",
            "qed_sampler_table", "qed_hist_photons", "qed_hist_leptons", "qed_field_advance",
            "qed_deposit_current", "qed_save_start", "qed_brems_init", "qed_brems_tables", "qed_step_brems",
            "qed_last_error"]

MLP_NPARAM = 34051
BREMS_NE, BREMS_NU = 256, 128
NOALLOC_MAX_LEPTONS = 524288
SAMPLER_TABLE, SAMPLER_MLP, SAMPLER_MLP_NBW = 0, 1, 2
NET_NCS, NET_NBW = 0, 1
DEPOSIT_BINNED, DEPOSIT_LOCAL = 0, 1

ALPHA = 1.0 / 137.035999084
XI_L = 2.42631023867e-6
A_E = 1.15965218128e-3


class QedError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [("xi_L", C.c_double), ("alpha", C.c_double), ("a_e", C.c_double), ("dt", C.c_double),
                ("p_max", C.c_double), ("seed", C.c_uint64), ("id_start", C.c_uint64),
                ("precision", C.c_int32), ("procs", C.c_uint32)]


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("circular", C.c_int32),
                ("a0", C.c_double), ("ncycles", C.c_double), ("phase0", C.c_double), ("pol_angle", C.c_double),
                ("w0", C.c_double), ("x_focus", C.c_double), ("phi_start", C.c_double),
                ("e0", C.c_double * 3), ("b0", C.c_double * 3), ("grid", C.c_void_p * 6),
                ("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("gx0", C.c_double), ("gy0", C.c_double)]


class Segment(C.Structure):
    _fields_ = [("begin", C.c_int64), ("end", C.c_int64), ("field", Field)]


AX_SLOPE_Y, AX_SLOPE_Z, AX_SLOPE_R, AX_ENERGY = 0, 1, 2, 3


class HistSpec(C.Structure):
    _fields_ = [("axis", C.c_int32 * 2), ("n", C.c_int32 * 2), ("lo", C.c_double * 2), ("hi", C.c_double * 2),
                ("pol_ref", C.c_double * 3)]


def hist_spec(axes, n, lo, hi, pol_ref=(0.0, 1.0, 0.0)) -> HistSpec:
    """Detector histogram axes (AX_*), bins, ranges (energy axes: log10 of the energy) and
    the lab vector that fixes the detector's polarisation basis."""
    h = HistSpec()
    for k in range(2):
        h.axis[k], h.n[k], h.lo[k], h.hi[k] = int(axes[k]), int(n[k]), float(lo[k]), float(hi[k])
    for k in range(3):
        h.pol_ref[k] = float(pol_ref[k])
    return h


class DepositSrc(C.Structure):
    _fields_ = [("leptons", C.c_void_p), ("x0", C.c_void_p * 3), ("n0", C.c_void_p)]


class FieldBC(C.Structure):
    _fields_ = [("open_x", C.c_int32), ("pad", C.c_int32), ("incoming", Field), ("gx0", C.c_double),
                ("gy0", C.c_double), ("t0", C.c_double)]


class Material(C.Structure):
    _fields_ = [("Z", C.c_int32), ("reserved", C.c_int32), ("n_atoms", C.c_double), ("x_lo", C.c_double),
                ("x_hi", C.c_double), ("k_cut", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("rate_lds", C.c_int32), ("ev_group", C.c_int32)]

    def as_dict(self):
        return {"blocks_per_cu": self.blocks_per_cu, "rate_lds": self.rate_lds, "ev_group": self.ev_group}


class CLeptons(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz", "id", "count")] + \
               [("capacity", C.c_int64), ("charge", C.c_int32)]


class CPhotons(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "y", "z", "kx", "ky", "kz", "w", "xi1", "xi2", "xi3",
                                          "e1x", "e1y", "e1z", "id", "alive", "count")] + \
               [("capacity", C.c_int64)]


_lib = None


def lib():
    """Load libqed.so; fails loudly if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise QedError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_11288_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, st = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "qed_init_tables": [C.POINTER(vp), vp, vp],
            "qed_destroy": [vp],
            "qed_gather": [vp, vp, C.c_int, vp, vp, i64, vp],
            "qed_push_spin": [vp, vp, C.c_int, vp, vp, i64, vp],
            "qed_push_radiative": [vp, vp, C.c_int, vp, C.c_uint32, i64, vp],
            "qed_hist_photons": [vp, vp, i64, vp, vp, vp],
            "qed_field_advance": [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, i64,
                                  vp],
            "qed_deposit_current": [vp, vp, C.c_int32, vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_double, vp],
            "qed_save_start": [vp, vp, vp, vp, vp],
            "qed_hist_leptons": [vp, vp, i64, vp, vp, vp],
            "qed_emit": [vp, vp, C.c_int, vp, vp, vp, i64, vp],
            "qed_step_leptons": [vp, vp, C.c_int, vp, vp, i64, vp],
            "qed_step_leptons_noalloc": [vp, vp, C.c_int, vp, vp, i64, vp],
            "qed_birefringence": [vp, vp, C.c_int, vp, i64, vp],
            "qed_pair": [vp, vp, C.c_int, vp, vp, vp, i64, vp],
            "qed_step_photons": [vp, vp, C.c_int, vp, vp, vp, i64, vp],
            "qed_step": [vp, vp, C.c_int, vp, vp, vp, i64, vp],
            "qed_compact_photons": [vp, vp, vp, vp],
            "qed_brems_init": [vp, vp, vp],
            "qed_brems_tables": [vp, vp, vp, vp],
            "qed_step_brems": [vp, vp, vp, i64, vp],
            "qed_sort_photons": [vp, vp, vp, vp, C.c_int32, vp],
            "qed_sort_leptons": [vp, vp, vp, vp, C.c_int32, vp],
            "qed_read_status": [vp, C.POINTER(C.c_uint32), vp],
            "qed_clear_status": [vp, vp],
            "qed_get_next_id": [vp, C.POINTER(C.c_uint64), vp],
            "qed_set_next_id": [vp, C.c_uint64, vp],
            "qed_table_export": [vp, C.c_int, vp, i64],
            "qed_set_step_events": [vp, vp],
            "qed_set_photon_events": [vp, vp],
            "qed_set_step_counter": [vp, vp],
            "qed_advance_step": [vp, i64, vp],
            "qed_get_tuning": [vp, vp],
            "qed_set_tuning": [vp, vp],
            "qed_autotune": [vp, vp, C.c_int, vp, i64, C.c_int, vp, vp],
            "qed_mlp_init": [vp, C.c_uint64, vp],
            "qed_mlp_set_params": [vp, vp, vp],
            "qed_mlp_get_params": [vp, vp, vp],
            "qed_mlp_samples": [vp, i64, C.c_uint64, vp, vp, vp],
            "qed_mlp_forward": [vp, vp, vp, i64, vp],
            "qed_mlp_gradient": [vp, vp, vp, i64, vp, vp, vp, vp],
            "qed_mlp_train_step": [vp, vp, vp, i64, vp, C.c_float, vp, vp],
            "qed_set_sampler": [vp, C.c_int],
            "qed_mlp_select": [vp, C.c_int],
            "qed_set_deposit_path": [vp, C.c_int],
            "qed_sampler_table": [vp, vp, vp, i64, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.restype = st
            f.argtypes = args
        L.qed_table_size.restype = i64
        L.qed_table_size.argtypes = [C.c_int]
        L.qed_last_error.restype = C.c_char_p
        L.qed_last_error.argtypes = [vp]
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------- buffers
LEPTON_KEYS = ("x", "y", "z", "px", "py", "pz", "w", "sx", "sy", "sz")
PHOTON_KEYS = ("x", "y", "z", "kx", "ky", "kz", "w", "xi1", "xi2", "xi3", "e1x", "e1y", "e1z")


class Leptons:
    """Device SoA electron or positron list (caller-owned memory)."""

    def __init__(self, capacity: int, charge: int, precision: int = QED_FP64, device="cuda"):
        torch = _torch()
        self.capacity, self.charge, self.precision = int(capacity), int(charge), precision
        sd = torch.float32 if precision == QED_MIXED else torch.float64
        for k in LEPTON_KEYS:
            setattr(self, k, torch.zeros(self.capacity, dtype=sd if k in ("sx", "sy", "sz") else torch.float64,
                                         device=device))
        self.id = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.count_t = torch.zeros(1, dtype=torch.int64, device=device)

    @classmethod
    def from_state(cls, st: dict, capacity=None, charge=-1, precision=QED_FP64, device="cuda"):
        torch = _torch()
        n = len(st["x"])
        L = cls(capacity or n, charge, precision, device)
        for k in LEPTON_KEYS:
            t = getattr(L, k)
            t[:n] = torch.as_tensor(np.ascontiguousarray(st[k]), dtype=t.dtype).to(device)
        L.id[:n] = torch.as_tensor(np.asarray(st["id"]).astype(np.uint64).view(np.int64)).to(device)
        L.count_t.fill_(n)
        return L

    @property
    def count(self) -> int:
        return int(self.count_t.item())

    def c(self) -> CLeptons:
        if getattr(self, "_c", None) is None:   # buffers never move: build the descriptor once
            s = CLeptons()
            for k in LEPTON_KEYS:
                setattr(s, k, getattr(self, k).data_ptr())
            s.id, s.count, s.capacity, s.charge = (self.id.data_ptr(), self.count_t.data_ptr(), self.capacity,
                                                   self.charge)
            self._c = s
        return self._c

    def to_numpy(self) -> dict:
        n = self.count
        out = {k: getattr(self, k)[:n].double().cpu().numpy() for k in LEPTON_KEYS}
        out["id"] = self.id[:n].cpu().numpy().view(np.uint64)
        return out


class Photons:
    """Device SoA photon list (caller-owned memory)."""

    def __init__(self, capacity: int, precision: int = QED_FP64, device="cuda"):
        torch = _torch()
        self.capacity, self.precision = int(capacity), precision
        sd = torch.float32 if precision == QED_MIXED else torch.float64
        for k in PHOTON_KEYS:
            low = k.startswith("xi") or k.startswith("e1")
            setattr(self, k, torch.zeros(self.capacity, dtype=sd if low else torch.float64, device=device))
        self.id = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.alive = torch.zeros(self.capacity, dtype=torch.uint8, device=device)
        self.count_t = torch.zeros(1, dtype=torch.int64, device=device)

    @classmethod
    def from_state(cls, st: dict, capacity=None, precision=QED_FP64, device="cuda"):
        torch = _torch()
        n = len(st["x"])
        G = cls(capacity or n, precision, device)
        for k in PHOTON_KEYS:
            t = getattr(G, k)
            t[:n] = torch.as_tensor(np.ascontiguousarray(st[k]), dtype=t.dtype).to(device)
        G.id[:n] = torch.as_tensor(np.asarray(st["id"]).astype(np.uint64).view(np.int64)).to(device)
        G.alive[:n] = torch.as_tensor(np.asarray(st.get("alive", np.ones(n, np.uint8)), dtype=np.uint8)).to(device)
        G.count_t.fill_(n)
        return G

    @property
    def count(self) -> int:
        return int(self.count_t.item())

    def c(self) -> CPhotons:
        if getattr(self, "_c", None) is None:
            s = CPhotons()
            for k in PHOTON_KEYS:
                setattr(s, k, getattr(self, k).data_ptr())
            s.id, s.alive, s.count, s.capacity = (self.id.data_ptr(), self.alive.data_ptr(), self.count_t.data_ptr(),
                                                  self.capacity)
            self._c = s
        return self._c

    def to_numpy(self) -> dict:
        n = self.count
        out = {k: getattr(self, k)[:n].double().cpu().numpy() for k in PHOTON_KEYS}
        out["id"] = self.id[:n].cpu().numpy().view(np.uint64)
        out["alive"] = self.alive[:n].cpu().numpy()
        return out


def make_field(spec: dict, keep: list | None = None) -> Field:
    """Field descriptor from a dict (same keys as the workload generators).  For GRID2D,
    spec['grid'] holds six float32 device tensors [ny][nx]."""
    f = Field()
    f.kind = int(spec.get("kind", FIELD_NONE))
    f.circular = int(spec.get("circular", 0))
    for k in ("a0", "ncycles", "phase0", "pol_angle", "w0", "x_focus", "phi_start", "dx", "dy", "gx0", "gy0"):
        setattr(f, k, float(spec.get(k, 0.0)))
    for i, v in enumerate(spec.get("e0", (0, 0, 0))):
        f.e0[i] = float(v)
    for i, v in enumerate(spec.get("b0", (0, 0, 0))):
        f.b0[i] = float(v)
    if f.kind == FIELD_GRID2D:
        f.nx, f.ny = int(spec["nx"]), int(spec["ny"])
        for c in range(6):
            g = spec["grid"][c]
            f.grid[c] = g.data_ptr()
            if keep is not None:
                keep.append(g)
    return f


def segments(specs) -> tuple:
    """[(begin, end, field_spec), ...] -> (ctypes array, n)."""
    specs = list(specs)
    arr = (Segment * len(specs))()
    keep = []
    for i, (b, e, fs) in enumerate(specs):
        arr[i].begin, arr[i].end = int(b), int(e)
        arr[i].field = make_field(fs, keep)
    arr._keep = keep
    return arr, len(specs)


def whole(field_spec: dict):
    """One segment covering every particle."""
    return segments([(0, 1 << 62, field_spec)])


# --------------------------------------------------------------------------- context
class Context:
    """A libqed context: device tables, constants, id counter, status word."""

    def __init__(self, *, dt, procs, seed, id_start, precision=QED_FP64, p_max=0.1, xi_L=XI_L, alpha=ALPHA,
                 a_e=A_E, stream=None):
        self.cfg = Config(xi_L, alpha, a_e, dt, p_max, seed, id_start, precision, procs)
        h = C.c_void_p()
        rc = lib().qed_init_tables(C.byref(h), C.byref(self.cfg), _stream(stream))
        if rc != QED_OK:
            raise QedError(f"qed_init_tables failed with status {rc}")
        self.h = h
        self.precision = precision

    def close(self):
        if getattr(self, "h", None):
            lib().qed_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, name):
        if rc != QED_OK:
            msg = lib().qed_last_error(self.h)
            raise QedError(f"{name}: status {rc}: {msg.decode() if msg else ''}")

    def gather(self, segs, L: Leptons, E6, step: int, stream=None):
        arr, n = segs
        self._check(lib().qed_gather(self.h, arr, n, C.byref(L.c()), _ptr(E6), step, _stream(stream)), "qed_gather")

    def push_spin(self, segs, L: Leptons, step: int, E6=None, stream=None):
        arr, n = segs
        self._check(lib().qed_push_spin(self.h, arr, n, C.byref(L.c()), _ptr(E6) if E6 is not None else None, step,
                                        _stream(stream)), "qed_push_spin")

    def push_radiative(self, segs, L: Leptons, mode: int, step: int, stream=None):
        """Push with radiation reaction: mode = RR_LL or RR_MLL, optionally | RR_RBMT."""
        arr, n = segs
        self._check(lib().qed_push_radiative(self.h, arr, n, C.byref(L.c()), int(mode), step, _stream(stream)),
                    "qed_push_radiative")

    def field_advance(self, grid: dict, dt: float, steps: int = 1, current=None, bc=None, stream=None):
        """Advance a GRID2D field (dict with 'grid' = six float32 device tensors [ny][nx],
        'nx', 'ny', 'dx', 'dy') in place by `steps` steps of the Yee solver, with the current
        `current` (three float32 device tensors [ny][nx]: Jx, Jy, Jz) if given.  bc: None
        (periodic) or a dict {'open_x': 1, 'incoming': pulse spec or None, 'gx0', 'gy0',
        't0'} for open x boundaries with a pulse entering through x_max."""
        arr = (C.c_void_p * 6)(*[g.data_ptr() for g in grid["grid"]])
        cur = None if current is None else (C.c_void_p * 3)(*[j.data_ptr() for j in current])
        b = None
        if bc is not None:
            b = FieldBC()
            b.open_x = int(bc.get("open_x", 1))
            if bc.get("incoming") is not None:
                b.incoming = make_field(bc["incoming"])
            b.gx0, b.gy0, b.t0 = float(bc.get("gx0", 0.0)), float(bc.get("gy0", 0.0)), float(bc.get("t0", 0.0))
        self._check(lib().qed_field_advance(self.h, arr, cur, C.byref(b) if b is not None else None, int(grid["nx"]),
                                            int(grid["ny"]), float(grid["dx"]), float(grid["dy"]), float(dt),
                                            int(steps), _stream(stream)), "qed_field_advance")

    def save_start(self, L: "Leptons", out=None, stream=None):
        """Positions and count of L at the start of a step, for deposit_current
        (qed_save_start): device tensors (x0, y0, z0, n0), written into `out` (a previous
        result) when given."""
        torch = _torch()
        if out is None:
            out = tuple(torch.empty(L.capacity, dtype=torch.float64, device=L.x.device) for _ in range(3)) + \
                (torch.zeros(1, dtype=torch.int64, device=L.x.device),)
        x0 = (C.c_void_p * 3)(*[t.data_ptr() for t in out[:3]])
        self._check(lib().qed_save_start(self.h, C.byref(L.c()), x0, _ptr(out[3]), _stream(stream)),
                    "qed_save_start")
        return out

    def set_deposit_path(self, path: int):
        """DEPOSIT_BINNED (any order) or DEPOSIT_LOCAL (lists kept in cell order) for later
        deposit_current calls (qed_set_deposit_path)."""
        self._check(lib().qed_set_deposit_path(self.h, int(path)), "qed_set_deposit_path")

    def deposit_current(self, sources, grid: dict, current, qscale: float, stream=None):
        """Add the current of the leptons of each source (L, start) that moved from the saved
        start positions to their current ones over one step of this context's dt to
        `current` (three float32 device tensors [ny][nx]); start = (x0, y0, z0, n0) as
        save_start returns them (float64 positions, int64 count).  One to four sources
        (electrons and positrons in one call cost one pass)."""
        arr = (DepositSrc * len(sources))()
        for k, (L, start) in enumerate(sources):
            arr[k].leptons = C.addressof(L.c())
            for c in range(3):
                arr[k].x0[c] = start[c].data_ptr()
            arr[k].n0 = start[3].data_ptr()
        cur = (C.c_void_p * 3)(*[j.data_ptr() for j in current])
        self._check(lib().qed_deposit_current(self.h, arr, len(sources), cur, int(grid["nx"]), int(grid["ny"]),
                                              float(grid["dx"]), float(grid["dy"]), float(grid["gx0"]),
                                              float(grid["gy0"]), float(self.cfg.dt), float(qscale), _stream(stream)),
                    "qed_deposit_current")

    def hist_photons(self, G: "Photons", begin: int, h: HistSpec, out=None, stream=None):
        """Add photons [begin, count) to a detector histogram [n1][n0][5] (float64 device
        tensor; allocated zeroed if not given) and return it."""
        torch = _torch()
        if out is None:
            out = torch.zeros((h.n[1], h.n[0], 5), dtype=torch.float64, device="cuda")
        self._check(lib().qed_hist_photons(self.h, C.byref(G.c()), int(begin), C.byref(h), _ptr(out),
                                           _stream(stream)), "qed_hist_photons")
        return out

    def hist_leptons(self, L: "Leptons", begin: int, h: HistSpec, out=None, stream=None):
        """The same for leptons (w, w gamma, w S)."""
        torch = _torch()
        if out is None:
            out = torch.zeros((h.n[1], h.n[0], 5), dtype=torch.float64, device="cuda")
        self._check(lib().qed_hist_leptons(self.h, C.byref(L.c()), int(begin), C.byref(h), _ptr(out),
                                           _stream(stream)), "qed_hist_leptons")
        return out

    def emit(self, segs, L: Leptons, E6, out: Photons | None, step: int, stream=None):
        arr, n = segs
        o = C.byref(out.c()) if out is not None else None
        self._check(lib().qed_emit(self.h, arr, n, C.byref(L.c()), _ptr(E6), o, step, _stream(stream)), "qed_emit")

    def step_leptons(self, segs, L: Leptons, out: Photons | None, step: int, stream=None):
        arr, n = segs
        o = C.byref(out.c()) if out is not None else None
        self._check(lib().qed_step_leptons(self.h, arr, n, C.byref(L.c()), o, step, _stream(stream)),
                    "qed_step_leptons")

    def step_leptons_noalloc(self, segs, L: Leptons, out: Photons | None, step: int, stream=None):
        arr, n = segs
        o = C.byref(out.c()) if out is not None else None
        self._check(lib().qed_step_leptons_noalloc(self.h, arr, n, C.byref(L.c()), o, step, _stream(stream)),
                    "qed_step_leptons_noalloc")

    def birefringence(self, segs, G: Photons, step: int, stream=None):
        arr, n = segs
        self._check(lib().qed_birefringence(self.h, arr, n, C.byref(G.c()), step, _stream(stream)),
                    "qed_birefringence")

    def pair(self, segs, G: Photons, em: Leptons | None, ep: Leptons | None, step: int, stream=None):
        arr, n = segs
        self._check(lib().qed_pair(self.h, arr, n, C.byref(G.c()), C.byref(em.c()) if em else None,
                                   C.byref(ep.c()) if ep else None, step, _stream(stream)), "qed_pair")

    def step_photons(self, segs, G: Photons, em: Leptons | None, ep: Leptons | None, step: int, stream=None):
        arr, n = segs
        self._check(lib().qed_step_photons(self.h, arr, n, C.byref(G.c()), C.byref(em.c()) if em else None,
                                           C.byref(ep.c()) if ep else None, step, _stream(stream)),
                    "qed_step_photons")

    def compact_photons(self, src: Photons, dst: Photons, stream=None):
        self._check(lib().qed_compact_photons(self.h, C.byref(src.c()), C.byref(dst.c()), _stream(stream)),
                    "qed_compact_photons")

    def brems_init(self, Z: int, n_atoms: float, x_lo: float, x_hi: float, k_cut: float, stream=None):
        """Bremsstrahlung tables of one target slab (atoms per (c / omega_L)^3; k_cut in m c^2)."""
        m = Material(Z, 0, n_atoms, x_lo, x_hi, k_cut)
        self._check(lib().qed_brems_init(self.h, C.byref(m), _stream(stream)), "qed_brems_init")

    def brems_tables(self, stream=None):
        """(sigma [256], cumulative rows [256, 128]) of the material, FP64 device tensors."""
        t = _torch()
        sig = t.empty(BREMS_NE, dtype=t.float64, device="cuda")
        cdf = t.empty((BREMS_NE, BREMS_NU), dtype=t.float64, device="cuda")
        self._check(lib().qed_brems_tables(self.h, _ptr(sig), _ptr(cdf), _stream(stream)), "qed_brems_tables")
        return sig, cdf

    def step_brems(self, em: Leptons, G: Photons, step: int, stream=None):
        self._check(lib().qed_step_brems(self.h, C.byref(em.c()), C.byref(G.c()), step, _stream(stream)),
                    "qed_step_brems")

    def sort_photons(self, src: Photons, dst: Photons, grid_spec: dict, bin_cells: int = 4, stream=None):
        """Live photons of src into dst, stably sorted by grid bin (dead ones dropped)."""
        f = make_field(grid_spec)
        self._check(lib().qed_sort_photons(self.h, C.byref(src.c()), C.byref(dst.c()), C.byref(f), bin_cells,
                                           _stream(stream)), "qed_sort_photons")

    def sort_leptons(self, src: Leptons, dst: Leptons, grid_spec: dict, bin_cells: int = 4, stream=None):
        """Leptons of src into dst, stably sorted by grid bin."""
        f = make_field(grid_spec)
        self._check(lib().qed_sort_leptons(self.h, C.byref(src.c()), C.byref(dst.c()), C.byref(f), bin_cells,
                                           _stream(stream)), "qed_sort_leptons")

    def read_status(self, stream=None) -> int:
        v = C.c_uint32()
        self._check(lib().qed_read_status(self.h, C.byref(v), _stream(stream)), "qed_read_status")
        return int(v.value)

    def clear_status(self, stream=None):
        self._check(lib().qed_clear_status(self.h, _stream(stream)), "qed_clear_status")

    def next_id(self, stream=None) -> int:
        v = C.c_uint64()
        self._check(lib().qed_get_next_id(self.h, C.byref(v), _stream(stream)), "qed_get_next_id")
        return int(v.value)

    def set_next_id(self, v: int, stream=None):
        self._check(lib().qed_set_next_id(self.h, int(v), _stream(stream)), "qed_set_next_id")

    def set_step_counter(self, counter=None):
        """Register a device int64 tensor (one element) whose value is added to the step of
        every later call (None unregisters); see advance_step."""
        if counter is not None:
            assert counter.dtype == _torch().int64 and counter.is_cuda and counter.numel() == 1
        self._counter = counter
        self._check(lib().qed_set_step_counter(self.h, _ptr(counter) if counter is not None else None),
                    "qed_set_step_counter")

    def advance_step(self, by: int = 1, stream=None):
        self._check(lib().qed_advance_step(self.h, int(by), _stream(stream)), "qed_advance_step")

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib().qed_get_tuning(self.h, C.byref(t)), "qed_get_tuning")
        return t.as_dict()

    def set_tuning(self, blocks_per_cu: int = 0, rate_lds: int = 0, ev_group: int = 8):
        t = Tuning(blocks_per_cu, rate_lds, ev_group)
        self._check(lib().qed_set_tuning(self.h, C.byref(t)), "qed_set_tuning")

    def autotune(self, segs, L: Leptons, step: int, reps: int = 3, stream=None) -> dict:
        arr, n = segs
        t = Tuning()
        self._check(lib().qed_autotune(self.h, arr, n, C.byref(L.c()), step, reps, C.byref(t), _stream(stream)),
                    "qed_autotune")
        return t.as_dict()

    # ---- learned sampler ------------------------------------------------------------
    def mlp_init(self, seed: int = 0, stream=None):
        self._check(lib().qed_mlp_init(self.h, int(seed), _stream(stream)), "qed_mlp_init")

    def mlp_set_params(self, params, stream=None):
        t = _torch()
        p = t.as_tensor(params, dtype=t.float32, device="cuda").contiguous()
        assert p.numel() == MLP_NPARAM
        self._check(lib().qed_mlp_set_params(self.h, _ptr(p), _stream(stream)), "qed_mlp_set_params")
        _torch().cuda.current_stream().synchronize()

    def mlp_get_params(self, stream=None):
        t = _torch()
        out = t.empty(MLP_NPARAM, dtype=t.float32, device="cuda")
        self._check(lib().qed_mlp_get_params(self.h, _ptr(out), _stream(stream)), "qed_mlp_get_params")
        return out

    def mlp_samples(self, n: int, seed: int, stream=None):
        t = _torch()
        X = t.empty((n, 4), dtype=t.float32, device="cuda")
        Y = t.empty((n, 3), dtype=t.float32, device="cuda")
        self._check(lib().qed_mlp_samples(self.h, n, int(seed), _ptr(X), _ptr(Y), _stream(stream)), "qed_mlp_samples")
        return X, Y

    def mlp_forward(self, X, Y=None, stream=None):
        t = _torch()
        n = X.shape[0]
        if Y is None:
            Y = t.empty((n, 3), dtype=t.float32, device="cuda")
        self._check(lib().qed_mlp_forward(self.h, _ptr(X), _ptr(Y), n, _stream(stream)), "qed_mlp_forward")
        return Y

    def mlp_gradient(self, X, T, w=(1.0, 1.0, 1.0), stream=None):
        t = _torch()
        g = t.empty(MLP_NPARAM, dtype=t.float32, device="cuda")
        loss = t.empty(1, dtype=t.float32, device="cuda")
        wa = (C.c_float * 3)(*w)
        self._check(lib().qed_mlp_gradient(self.h, _ptr(X), _ptr(T), X.shape[0], wa, _ptr(g), _ptr(loss),
                                           _stream(stream)), "qed_mlp_gradient")
        return loss, g

    def mlp_train_step(self, X, T, lr: float, w=(1.0, 1.0, 1.0), loss=None, stream=None):
        t = _torch()
        if loss is None:
            loss = t.empty(1, dtype=t.float32, device="cuda")
        wa = (C.c_float * 3)(*w)
        self._check(lib().qed_mlp_train_step(self.h, _ptr(X), _ptr(T), X.shape[0], wa, C.c_float(lr), _ptr(loss),
                                             _stream(stream)), "qed_mlp_train_step")
        return loss

    def sampler_table(self, X, Y=None, stream=None):
        t = _torch()
        if Y is None:
            Y = t.empty((X.shape[0], 3), dtype=t.float32, device="cuda")
        self._check(lib().qed_sampler_table(self.h, _ptr(X), _ptr(Y), X.shape[0], _stream(stream)),
                    "qed_sampler_table")
        return Y

    def mlp_select(self, net: int):
        """The network later mlp_* / sampler_table calls act on: NET_NCS or NET_NBW."""
        self._check(lib().qed_mlp_select(self.h, int(net)), "qed_mlp_select")

    def mlp_load_pretrained(self, path: str | None = None, net: int | None = None):
        """Parameters of a network shipped with the package into that network (the selected
        one if net is None; the selection is left at net): sampler_ncs.npy, trained by
        `python -m paper_2306_11288_amd.train_sampler --samples 50000000 --epochs 2
        --batch 4096 --seed 0`; sampler_nbw.npy, by `python -m
        paper_2306_11288_amd.train_sampler --net nbw --samples 50000000 --epochs 4 --batch
        4096 --seed 0`; or another .npy file."""
        if net is not None:
            self.mlp_select(net)
        name = "sampler_nbw.npy" if net == NET_NBW else "sampler_ncs.npy"
        p = np.load(path or os.path.join(_HERE, name), allow_pickle=False)
        self.mlp_set_params(p.astype(np.float32))

    def set_sampler(self, sampler: int):
        """SAMPLER_TABLE, or the bits SAMPLER_MLP (NCS emissions) and SAMPLER_MLP_NBW (pair
        creations) for the learned samplers (qed_set_sampler)."""
        self._check(lib().qed_set_sampler(self.h, int(sampler)), "qed_set_sampler")

    def set_step_events(self, events=None):
        """Record four torch.cuda.Event around the decide / scan / event kernels of every
        later NCS lepton step (None switches it off); the events must outlive their use."""
        if events is None:
            self._check(lib().qed_set_step_events(self.h, None), "qed_set_step_events")
            return
        for e in events:   # torch creates the HIP event on its first record
            if not e.cuda_event:
                e.record()
        arr = (C.c_void_p * 4)(*[C.c_void_p(e.cuda_event) for e in events])
        self._check(lib().qed_set_step_events(self.h, arr), "qed_set_step_events")

    def set_photon_events(self, events=None):
        """Record two torch.cuda.Event around the photon kernels of every later photon
        stage (None switches it off); the events must outlive their use."""
        if events is None:
            self._check(lib().qed_set_photon_events(self.h, None), "qed_set_photon_events")
            return
        for e in events:
            if not e.cuda_event:
                e.record()
        arr = (C.c_void_p * 2)(*[C.c_void_p(e.cuda_event) for e in events])
        self._check(lib().qed_set_photon_events(self.h, arr), "qed_set_photon_events")

    def table_export(self, which: int) -> np.ndarray:
        n = lib().qed_table_size(which)
        out = np.zeros(n)
        self._check(lib().qed_table_export(self.h, which, out.ctypes.data_as(C.c_void_p), n), "qed_table_export")
        return out

    def step(self, segs, em: Leptons | None, ep: Leptons | None, G: Photons | None, step: int, stream=None):
        """One whole step with the result of the Spin-QED chain (qed_step)."""
        arr, n = segs
        self._check(lib().qed_step(self.h, arr, n, C.byref(em.c()) if em else None,
                                   C.byref(ep.c()) if ep else None, C.byref(G.c()) if G else None, step,
                                   _stream(stream)), "qed_step")

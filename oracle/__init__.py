"""CPU oracle of lumped-element tracking (ctypes binding of liboracle.so).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path (``paper_1710_07350_amd``); the two meet only in the
seeded input descriptions of ``paper_1710_07350_amd.inputs``, which hold no
tracking arithmetic.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None

KIND = {"EDRIFT": 1, "QUAD": 2, "MAP2": 3, "MULT": 4, "KQUAD": 5, "CSBEND": 6,
        "RFCA": 7, "WAKE": 8, "RADKICK": 9, "MARKER": 10, "TRWAKE": 11, "MAP3": 12}
APER = {"NONE": 0, "RECT": 1, "ELLIPSE": 2}
TAG_RAD = 2


class OrcElem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("aper", C.c_int32), ("order", C.c_int32),
                ("nsteps", C.c_int32), ("nbins", C.c_int32), ("pad", C.c_int32),
                ("L", C.c_double), ("k", C.c_double), ("angle", C.c_double),
                ("volt", C.c_double), ("phase", C.c_double), ("freq", C.c_double),
                ("wake_A", C.c_double), ("wake_tau0", C.c_double),
                ("wake_omega", C.c_double), ("charge", C.c_double),
                ("sigma", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
                ("coef", C.c_double * 504)]


class OrcBeam(C.Structure):
    _fields_ = [("z", C.POINTER(C.c_double) * 6), ("id", C.POINTER(C.c_uint32)),
                ("lost_at", C.POINTER(C.c_int64)), ("n", C.c_int64), ("n0", C.c_int64)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        d, u32, u64, i32, i64 = C.c_double, C.c_uint32, C.c_uint64, C.c_int32, C.c_int64
        pd = C.POINTER(C.c_double)
        pu32 = C.POINTER(C.c_uint32)
        for f in ("orc_sin", "orc_cos", "orc_log", "orc_exp"):
            getattr(L, f).restype = d
            getattr(L, f).argtypes = [d]
        L.orc_philox4x32_10.argtypes = [pu32, pu32, pu32]
        L.orc_gauss.restype = d
        L.orc_gauss.argtypes = [u32, u32, u32, u64]
        L.orc_quad_coef.argtypes = [d, d, pd]
        L.orc_yoshida.argtypes = [pd, pd]
        L.orc_quad3_coef.argtypes = [d, d, pd]
        L.orc_track.restype = i64
        L.orc_track.argtypes = [C.POINTER(OrcBeam), C.POINTER(OrcElem), i32, i32, i32, d, u64, pd]
        L.orc_histogram.argtypes = [pd, C.POINTER(C.c_int64), i64, i32, pd, pu32]
        L.orc_wake_table.argtypes = [d, d, i32, d, d, pd]
        L.orc_convolve.argtypes = [pu32, pd, i32, pd]
        L.orc_wake_kick.argtypes = [C.POINTER(OrcBeam), pd, pd, i32, d]
        pi64 = C.POINTER(C.c_int64)
        L.orc_dipole_quantum.restype = i64
        L.orc_dipole_quantum.argtypes = [d]
        L.orc_dipole_histogram.argtypes = [pd, pd, pd, pi64, i64, i32, pd, pu32, pi64, pi64]
        L.orc_dipole_metres.argtypes = [pi64, i32, pd]
        L.orc_trwake_table.argtypes = [d, d, i32, d, d, pd]
        L.orc_convolve_f64.argtypes = [pd, pd, i32, pd]
        L.orc_trwake_kick.argtypes = [C.POINTER(OrcBeam), pd, pd, pd, i32, d]
        L.orc_moments.argtypes = [C.POINTER(OrcBeam), pd]
        L.orc_compact.restype = i64
        L.orc_compact.argtypes = [C.POINTER(OrcBeam)]
        L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32
        _LIB = L
    return _LIB


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- scalars
def sin(x: float) -> float: return lib().orc_sin(x)
def cos(x: float) -> float: return lib().orc_cos(x)
def log(x: float) -> float: return lib().orc_log(x)
def exp(x: float) -> float: return lib().orc_exp(x)


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (C.c_uint32 * 4)(*[v & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[v & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def gauss(pid: int, step: int, tag: int, seed: int) -> float:
    return lib().orc_gauss(pid, step, tag, seed)


def quad_coef(L: float, k1: float) -> np.ndarray:
    out = np.zeros(168)
    lib().orc_quad_coef(L, k1, _ptr(out, C.c_double))
    return out


def quad3_coef(L: float, k1: float) -> np.ndarray:
    out = np.zeros(504)
    lib().orc_quad3_coef(L, k1, _ptr(out, C.c_double))
    return out


def yoshida():
    c = np.zeros(4)
    d = np.zeros(3)
    lib().orc_yoshida(_ptr(c, C.c_double), _ptr(d, C.c_double))
    return c, d


def set_threads(n: int) -> None: lib().orc_set_threads(n)
def get_threads() -> int: return lib().orc_get_threads()


# ---------------------------------------------------------------- beams
class Beam:
    """Host beam: z[6][n] float64, id uint32, lost_at int64 (numpy, owned)."""

    def __init__(self, z, pid, lost_at, n0: Optional[int] = None):
        self.z = np.ascontiguousarray(z, dtype=np.float64).copy()
        self.id = np.ascontiguousarray(pid, dtype=np.uint32).copy()
        self.lost_at = np.ascontiguousarray(lost_at, dtype=np.int64).copy()
        self.n0 = int(n0 if n0 is not None else self.z.shape[1])

    @classmethod
    def from_inputs(cls, d: dict, n0: Optional[int] = None) -> "Beam":
        return cls(d["z"], d["id"], d["lost_at"], n0)

    @property
    def n(self) -> int:
        return self.z.shape[1]

    def cstruct(self) -> OrcBeam:
        b = OrcBeam()
        for k in range(6):
            b.z[k] = self.z[k].ctypes.data_as(C.POINTER(C.c_double))
        b.id = _ptr(self.id, C.c_uint32)
        b.lost_at = _ptr(self.lost_at, C.c_int64)
        b.n = self.n
        b.n0 = self.n0
        return b


def elements(lattice) -> "C.Array":
    arr = (OrcElem * max(1, len(lattice)))()
    for i, e in enumerate(lattice):
        r = arr[i]
        r.kind = KIND[e.kind]
        r.aper = APER[e.aperture]
        r.order, r.nsteps, r.nbins = e.order, e.nsteps, e.nbins
        r.L, r.k, r.angle = e.L, e.k, e.angle
        r.volt, r.phase, r.freq = e.volt, e.phase, e.freq
        r.wake_A, r.wake_tau0, r.wake_omega, r.charge = e.wake_A, e.wake_tau0, e.wake_omega, e.charge
        r.sigma, r.ax, r.ay = e.sigma, e.ax, e.ay
        if e.coef is not None:
            for j in range(len(e.coef)):
                r.coef[j] = float(e.coef[j])
    return arr


def track(beam: Beam, lattice, passes: int, first_pass: int = 0, p_ref: float = 1e9,
          seed: int = 0, moments: bool = False):
    """Track in place; returns (n_alive, moments[passes][28] or None)."""
    arr = elements(lattice)
    mom = np.zeros((passes, 28)) if moments else None
    cb = beam.cstruct()
    n = lib().orc_track(C.byref(cb), arr, len(lattice), passes, first_pass, p_ref, seed,
                        _ptr(mom, C.c_double) if mom is not None else None)
    return int(n), mom


def histogram(s, lost_at, nbins: int):
    s = np.ascontiguousarray(s, dtype=np.float64)
    la = np.ascontiguousarray(lost_at, dtype=np.int64)
    rng = np.zeros(2)
    cnt = np.zeros(nbins, dtype=np.uint32)
    lib().orc_histogram(_ptr(s, C.c_double), _ptr(la, C.c_int64), len(s), nbins,
                        _ptr(rng, C.c_double), _ptr(cnt, C.c_uint32))
    return rng, cnt


def wake_table(smin: float, smax: float, nbins: int, tau0: float, omega: float):
    w = np.zeros(nbins)
    lib().orc_wake_table(smin, smax, nbins, tau0, omega, _ptr(w, C.c_double))
    return w


def convolve(counts, w):
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    v = np.zeros(len(w))
    lib().orc_convolve(_ptr(counts, C.c_uint32), _ptr(w, C.c_double), len(w), _ptr(v, C.c_double))
    return v


def wake_kick(beam: Beam, rng, v, kfac: float) -> None:
    rng = np.ascontiguousarray(rng, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    cb = beam.cstruct()
    lib().orc_wake_kick(C.byref(cb), _ptr(rng, C.c_double), _ptr(v, C.c_double), len(v), kfac)


# ---------------------------------------------------------------- transverse wake
def dipole_quantum(x: float) -> int:
    """x as an integer multiple of 2^-40 m (clamped to 1 m, ties to even)."""
    return int(lib().orc_dipole_quantum(x))


def dipole_histogram(s, x, y, lost_at, nbins: int):
    """(range, counts, dx, dy): the histogram of s and the per-bin sums of
    the quantised x and y (int64, units of 2^-40 m)."""
    s, x, y = (np.ascontiguousarray(a, dtype=np.float64) for a in (s, x, y))
    la = np.ascontiguousarray(lost_at, dtype=np.int64)
    rng = np.zeros(2)
    cnt = np.zeros(nbins, dtype=np.uint32)
    dx = np.zeros(nbins, dtype=np.int64)
    dy = np.zeros(nbins, dtype=np.int64)
    lib().orc_dipole_histogram(_ptr(s, C.c_double), _ptr(x, C.c_double), _ptr(y, C.c_double),
                               _ptr(la, C.c_int64), len(s), nbins, _ptr(rng, C.c_double),
                               _ptr(cnt, C.c_uint32), _ptr(dx, C.c_int64), _ptr(dy, C.c_int64))
    return rng, cnt, dx, dy


def dipole_metres(d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.int64)
    out = np.zeros(len(d))
    lib().orc_dipole_metres(_ptr(d, C.c_int64), len(d), _ptr(out, C.c_double))
    return out


def trwake_table(smin: float, smax: float, nbins: int, tau0: float, omega: float):
    w = np.zeros(nbins)
    lib().orc_trwake_table(smin, smax, nbins, tau0, omega, _ptr(w, C.c_double))
    return w


def convolve_f64(c, w):
    c = np.ascontiguousarray(c, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    v = np.zeros(len(w))
    lib().orc_convolve_f64(_ptr(c, C.c_double), _ptr(w, C.c_double), len(w), _ptr(v, C.c_double))
    return v


def trwake_kick(beam: Beam, rng, vx, vy, kfac: float) -> None:
    rng = np.ascontiguousarray(rng, dtype=np.float64)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    cb = beam.cstruct()
    lib().orc_trwake_kick(C.byref(cb), _ptr(rng, C.c_double), _ptr(vx, C.c_double),
                          _ptr(vy, C.c_double), len(vx), kfac)


def moments(beam: Beam) -> np.ndarray:
    out = np.zeros(28)
    cb = beam.cstruct()
    lib().orc_moments(C.byref(cb), _ptr(out, C.c_double))
    return out


def compact(beam: Beam) -> int:
    cb = beam.cstruct()
    return int(lib().orc_compact(C.byref(cb)))


def wake_kfac(charge: float, n0: int, A: float, p_ref: float) -> float:
    """Energy-kick factor ((Q/N0) A)/P of the wake step."""
    return ((charge / float(n0)) * A) / p_ref

"""Seeded synthetic inputs: beams and lattice descriptions.

This module is shared by the CPU oracle and the HIP path as their common
*input*.  It holds none of the tracking method's arithmetic: beams are drawn
with numpy's PCG64 generator, and a lattice is a list of `Element`
descriptions carrying only physical parameters (lengths, strengths,
voltages, apertures).  Each side turns a description into its own element
records, transfer-map coefficients and integrator constants.

Workloads (the paper's own LCLS lattice and regression suite are not
available; these synthetic beams and lattices stand in for them):

* ``fodo``   -- 10 FODO cells of exact drifts, second-order thick quads and
  thin sextupoles, 5 mm rectangular aperture after every element.
* ``bc``     -- linac bunch compressor: 8 zero-length RF cavities, each
  followed by the longitudinal wake step, then a second-order chicane map.
* ``ring``   -- 40-cell storage ring of kick-drift quads, sector bends and
  random thin sextupoles, an elliptical aperture and a once-per-turn Gaussian
  energy kick.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Element kinds (names follow the beamline element names of the paper's
# element table: EDRIFT, QUAD matrix, thin multipole, KQUAD, CSBEND, RFCA,
# WAKE, TRWAKE; MAP2 is an explicit second-order transport map, RADKICK the
# random energy kick).
KINDS = ("EDRIFT", "QUAD", "MAP2", "MULT", "KQUAD", "CSBEND", "RFCA", "WAKE",
         "RADKICK", "MARKER", "TRWAKE", "MAP3")
APERTURES = ("NONE", "RECT", "ELLIPSE")

C_LIGHT = 299792458.0


@dataclasses.dataclass
class Element:
    kind: str
    L: float = 0.0            # length [m]
    k: float = 0.0            # K1 [m^-2] (QUAD/KQUAD) or KnL [m^-n] (MULT)
    order: int = 0            # MULT order n (1 quad, 2 sext, 3 oct); QUAD: 3 = third-order map
    nsteps: int = 1           # Yoshida-4 steps (KQUAD/CSBEND)
    angle: float = 0.0        # bend angle [rad] (CSBEND)
    volt: float = 0.0         # RF voltage [V]
    phase: float = 0.0        # RF phase [rad], cosine convention, crest at 0
    freq: float = 0.0         # RF frequency [Hz]
    wake_A: float = 0.0       # resonator wake amplitude [V/C] (TRWAKE: [V/(C m)])
    wake_tau0: float = 0.0    # decay time [s]
    wake_omega: float = 0.0   # angular frequency [rad/s]
    charge: float = 0.0       # bunch charge [C]
    nbins: int = 0            # histogram bins (WAKE, TRWAKE)
    sigma: float = 0.0        # RADKICK rms energy kick
    coef: Optional[np.ndarray] = None  # MAP2: 168 doubles C[6], R[6][6], T[6][21]; MAP3: + U[6][56]
    aperture: str = "NONE"
    ax: float = 0.0           # RECT half-width x / ELLIPSE semi-axis a [m]
    ay: float = 0.0           # RECT half-width y / ELLIPSE semi-axis b [m]

    def __post_init__(self):
        assert self.kind in KINDS, self.kind
        assert self.aperture in APERTURES, self.aperture


# --------------------------------------------------------------------------
# beams
# --------------------------------------------------------------------------
BEAM_SIGMAS = (1e-3, 1e-4, 1e-3, 1e-4, 1e-3, 1e-3)   # x, x', y, y', s, delta


def gaussian_beam(n: int, seed: int = 0, sigmas: Sequence[float] = BEAM_SIGMAS,
                  chirp: float = 0.0) -> dict:
    """Independent Gaussian coordinates, ids 0..n-1, all particles alive.

    `chirp` h adds the linear energy-position correlation delta += h*s of the
    bunch-compressor workload (h = -10 m^-1) to the drawn coordinates.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((6, n))
    for k in range(6):
        z[k] *= sigmas[k]
    if chirp != 0.0:
        z[5] += chirp * z[4]
    return {
        "z": np.ascontiguousarray(z, dtype=np.float64),
        "id": np.arange(n, dtype=np.uint32),
        "lost_at": np.full(n, -1, dtype=np.int64),
    }


def uniform_box_beam(n: int, seed: int, half_widths: Sequence[float]) -> dict:
    """Uniform 6D box of the given half widths (surrogate training data)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.uniform(-1.0, 1.0, size=(6, n))
    for k in range(6):
        z[k] *= half_widths[k]
    return {"z": np.ascontiguousarray(z), "id": np.arange(n, dtype=np.uint32),
            "lost_at": np.full(n, -1, dtype=np.int64)}


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------
def fodo_lattice(ncells: int = 10, k1: float = 1.2, k2l: float = 5.0,
                 aper: float = 5e-3, quad_order: int = 2) -> List[Element]:
    """10 FODO cells [D 1 m, QF 0.2 m, SF, D 1 m, QD 0.2 m, SD] with the
    aperture |x|,|y| < 5 mm after every element (60 elements per pass);
    quad_order 3 tracks the quadrupoles with their third-order maps."""
    a = dict(aperture="RECT", ax=aper, ay=aper)
    qo = 3 if quad_order == 3 else 0
    cell = [
        Element("EDRIFT", L=1.0, **a),
        Element("QUAD", L=0.2, k=+k1, order=qo, **a),
        Element("MULT", k=+k2l, order=2, **a),
        Element("EDRIFT", L=1.0, **a),
        Element("QUAD", L=0.2, k=-k1, order=qo, **a),
        Element("MULT", k=-k2l, order=2, **a),
    ]
    return [dataclasses.replace(e) for _ in range(ncells) for e in cell]


def chicane_coef(r56: float = -0.05, t566: float = 0.075) -> np.ndarray:
    """Explicit second-order chicane map: identity plus R56 and T566.

    Layout: C[6], R[6][6] row-major, T[6][21] with the pair index of (j,k),
    j<=k, running (0,0),(0,1),...,(0,5),(1,1),...,(5,5).
    """
    c = np.zeros(168)
    R = c[6:42].reshape(6, 6)
    for i in range(6):
        R[i, i] = 1.0
    R[4, 5] = r56
    T = c[42:].reshape(6, 21)
    T[4, 20] = t566          # pair (5,5) is the last of the 21 pairs
    return c


BC_P0_EV = 100e6
BC_CHIRP = -10.0


def bc_lattice(ncav: int = 8, volt: float = 20e6, phase_deg: float = -20.0,
               freq: float = 1.3e9, nbins: int = 1024, fp_mode: str = "fp32") -> List[Element]:
    """8 x [RFCA, WAKE] then the chicane MAP2 (one pass)."""
    phase = math.radians(phase_deg)
    out: List[Element] = []
    for _ in range(ncav):
        out.append(Element("RFCA", volt=volt, phase=phase, freq=freq))
        out.append(Element("WAKE", wake_A=1e14, wake_tau0=10e-12,
                           wake_omega=2.0 * math.pi * 50e9, charge=1e-9,
                           nbins=nbins))
    out.append(Element("MAP2", coef=chicane_coef()))
    return out


def rfcw_lattice(ncav: int = 8, volt: float = 20e6, phase_deg: float = -20.0,
                 freq: float = 1.3e9, nbins: int = 1024, trans_A: float = 1e16) -> List[Element]:
    """The bunch compressor with the transverse wake of each cavity: 8 x
    [RFCA, WAKE, TRWAKE] then the chicane (the RF-cavity-with-wakes element
    of the paper's element table, split into its parts)."""
    phase = math.radians(phase_deg)
    out: List[Element] = []
    for _ in range(ncav):
        out.append(Element("RFCA", volt=volt, phase=phase, freq=freq))
        out.append(Element("WAKE", wake_A=1e14, wake_tau0=10e-12,
                           wake_omega=2.0 * math.pi * 50e9, charge=1e-9, nbins=nbins))
        out.append(Element("TRWAKE", wake_A=trans_A, wake_tau0=10e-12,
                           wake_omega=2.0 * math.pi * 50e9, charge=1e-9, nbins=nbins))
    out.append(Element("MAP2", coef=chicane_coef()))
    return out


def ring_sextupoles(seed: int, n: int = 80, lim: float = 10.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    return rng.uniform(-lim, lim, size=n)


def ring_lattice(seed: int = 0, ncells: int = 40, k1: float = 0.8,
                 sext: Optional[np.ndarray] = None, radiation: float = 1e-5,
                 aper=(10e-3, 5e-3), nsteps: int = 1) -> List[Element]:
    """40 cells [QF 0.3, SF, D 0.5, B 1.5, D 0.5, QD 0.3, SD, D 0.5, B, D 0.5]
    with an elliptical aperture after every magnet element, then one
    RADKICK per turn (401 elements per turn)."""
    if sext is None:
        sext = ring_sextupoles(seed, 2 * ncells)
    a = dict(aperture="ELLIPSE", ax=aper[0], ay=aper[1])
    theta = 2.0 * math.pi / (2 * ncells)
    out: List[Element] = []
    for c in range(ncells):
        out += [
            Element("KQUAD", L=0.3, k=+k1, nsteps=nsteps, **a),
            Element("MULT", k=float(sext[2 * c]), order=2, **a),
            Element("EDRIFT", L=0.5, **a),
            Element("CSBEND", L=1.5, angle=theta, nsteps=nsteps, **a),
            Element("EDRIFT", L=0.5, **a),
            Element("KQUAD", L=0.3, k=-k1, nsteps=nsteps, **a),
            Element("MULT", k=float(sext[2 * c + 1]), order=2, **a),
            Element("EDRIFT", L=0.5, **a),
            Element("CSBEND", L=1.5, angle=theta, nsteps=nsteps, **a),
            Element("EDRIFT", L=0.5, **a),
        ]
    if radiation > 0.0:
        out.append(Element("RADKICK", sigma=radiation))
    return out


def batch_variant_sizes(nvar: int = 256, seed: int = 0, lo: float = 1e3,
                        hi: float = 1e5) -> np.ndarray:
    """Particle counts log-uniform in [lo, hi] for the batched scan."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    u = rng.uniform(0.0, 1.0, size=nvar)
    return np.floor(lo * (hi / lo) ** u).astype(np.int64)


# --------------------------------------------------------------------------
# surrogate network: initial weights
# --------------------------------------------------------------------------
MLP_SHAPES = [("W1", (256, 6)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (256, 256)), ("b3", (256,)), ("W4", (6, 256)), ("b4", (6,))]


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded initial parameter vector (FP32, layout W1, b1, ..., W4, b4 with
    W[out][in]): weights uniform in +-1/sqrt(fan_in) (PCG64([seed, 5])),
    biases zero; the s column of W1 and the delta row of W4 are zero and W4 is
    scaled by 0.1."""
    rng = np.random.Generator(np.random.PCG64([seed, 5]))
    parts = []
    for name, shp in MLP_SHAPES:
        if name.startswith("W"):
            lim = 1.0 / math.sqrt(shp[1])
            a = rng.uniform(-lim, lim, size=shp).astype(np.float32)
            if name == "W1":
                a[:, 4] = 0.0
            if name == "W4":
                a[5, :] = 0.0
                a *= np.float32(0.1)
        else:
            a = np.zeros(shp, dtype=np.float32)
        parts.append(a.reshape(-1))
    return np.concatenate(parts)


def workload(name: str):
    """(lattice, beam kwargs, passes, p_ref) of a named workload."""
    if name == "fodo":
        return fodo_lattice(), dict(n=10_000, seed=0), 100, 1e9
    if name == "bc":
        return bc_lattice(), dict(n=4_000_000, seed=0, chirp=BC_CHIRP), 1, BC_P0_EV
    if name == "ring":
        return ring_lattice(0), dict(n=1_000_000, seed=0), 1000, 1e9
    raise KeyError(name)

"""Thin ctypes binding of libtrk.so (include/trk.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the computation runs in the library's kernels.  The
binding refuses to run when the library is missing -- there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrk.so")

TRK_OK, TRK_EINVAL, TRK_EPTR, TRK_EHIP, TRK_ENOMEM, TRK_ERANGE = 0, -1, -2, -3, -4, -5
KIND = {"EDRIFT": 1, "QUAD": 2, "MAP2": 3, "MULT": 4, "KQUAD": 5, "CSBEND": 6,
        "RFCA": 7, "WAKE": 8, "RADKICK": 9, "MARKER": 10, "TRWAKE": 11, "MAP3": 12}
APER = {"NONE": 0, "RECT": 1, "ELLIPSE": 2}
WAKE_FP64, WAKE_FP32_MFMA = 0, 1
MAX_BINS = 4096

# symbols declared in include/trk.h
EXPORTS = ("trk_lattice_create", "trk_lattice_destroy", "trk_workspace_size", "trk_track",
           "trk_histogram", "trk_wake_convolve", "trk_wake_kick", "trk_dipole_histogram",
           "trk_trwake_convolve", "trk_trwake_kick", "trk_moments", "trk_moments_noalloc", "trk_moments_compensated",
           "trk_compact_lost", "trk_compact_lost_mode", "trk_elementary", "trk_philox4x32_10", "trk_gauss",
           "trk_probe_stream", "trk_probe_fma",
           "trk_status_string", "trk_last_error", "trk_profile_enable", "trk_profile_read",
           "trk_batch_create", "trk_batch_destroy", "trk_batch_workspace_size",
           "trk_track_batched", "trk_mlp_create", "trk_mlp_destroy", "trk_mlp_get_params",
           "trk_mlp_forward", "trk_mlp_workspace_size", "trk_mlp_backward", "trk_mlp_adam_step",
           "trk_mlp_train", "trk_surrogate_create", "trk_surrogate_destroy",
           "trk_surrogate_get_info", "trk_surrogate_workspace_size", "trk_surrogate_gate",
           "trk_surrogate_sample", "trk_surrogate_pairs", "trk_surrogate_fit_scale",
           "trk_surrogate_apply")
MLP_NPARAM = 134918
MLP_BF16, MLP_BF16X2 = 0, 1


class TrkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"trk error {status}: {msg}")
        self.status = status


class Element(C.Structure):
    _fields_ = [("kind", C.c_int32), ("aperture", C.c_int32), ("order", C.c_int32),
                ("nsteps", C.c_int32), ("nbins", C.c_int32), ("reserved", C.c_int32),
                ("L", C.c_double), ("k", C.c_double), ("angle", C.c_double),
                ("volt", C.c_double), ("phase", C.c_double), ("freq", C.c_double),
                ("wake_A", C.c_double), ("wake_tau0", C.c_double), ("wake_omega", C.c_double),
                ("charge", C.c_double), ("sigma", C.c_double), ("ax", C.c_double),
                ("ay", C.c_double), ("coef", C.POINTER(C.c_double))]


class BeamStruct(C.Structure):
    _fields_ = [("x", C.c_void_p), ("xp", C.c_void_p), ("y", C.c_void_p), ("yp", C.c_void_p),
                ("s", C.c_void_p), ("dp", C.c_void_p), ("id", C.c_void_p),
                ("lost_at", C.c_void_p), ("n_alive", C.c_void_p), ("n_total", C.c_int64)]


class Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first_pass", C.c_int32),
                ("passes_per_launch", C.c_int32), ("max_elems_per_launch", C.c_int32),
                ("wake_mode", C.c_int32), ("run_ppt", C.c_int32), ("run_blocks", C.c_int32),
                ("run_longit", C.c_int32), ("run_nt", C.c_int32), ("run_hist", C.c_int32),
                ("p_ref_eV", C.c_double), ("moments", C.c_void_p)]


class BatchTuning(C.Structure):
    _fields_ = [("ppt", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("passes_per_launch", C.c_int32), ("use_graph", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("precision", C.c_int32),
                ("reserved", C.c_int32), ("lr0", C.c_double), ("lr_min", C.c_double),
                ("seed", C.c_uint64)]


class SurrOpts(C.Structure):
    _fields_ = [("half_width", C.c_double * 6), ("margin", C.c_double), ("h_rel", C.c_double),
                ("aper_a", C.c_double), ("aper_b", C.c_double)]


class SurrInfo(C.Structure):
    _fields_ = [("C", C.c_double * 6), ("R", C.c_double * 36), ("D", C.c_double * 6),
                ("alpha_x", C.c_double), ("beta_x", C.c_double), ("gamma_x", C.c_double),
                ("eta", C.c_double), ("etap", C.c_double), ("alpha_y", C.c_double),
                ("beta_y", C.c_double), ("gamma_y", C.c_double), ("beta_hat_x", C.c_double),
                ("beta_hat_y", C.c_double), ("eta_hat", C.c_double), ("lim", C.c_double),
                ("sample_half_width", C.c_double * 6)]


class Wake(C.Structure):
    _fields_ = [("A", C.c_double), ("tau0", C.c_double), ("omega", C.c_double),
                ("charge", C.c_double)]


_LIB = None


def lib():
    """Load libtrk.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, d, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32,
                                         C.c_uint64, C.c_double, C.c_size_t)
        L.trk_lattice_create.argtypes = [C.POINTER(Element), i32, C.POINTER(vp)]
        L.trk_lattice_destroy.argtypes = [vp]
        L.trk_lattice_destroy.restype = None
        L.trk_workspace_size.argtypes = [vp, i64]
        L.trk_workspace_size.restype = sz
        L.trk_track.argtypes = [C.POINTER(BeamStruct), vp, i32, C.POINTER(Opts), vp, sz, vp]
        L.trk_histogram.argtypes = [C.POINTER(BeamStruct), i32, vp, vp, vp, sz, vp]
        L.trk_wake_convolve.argtypes = [vp, i32, vp, d, d, i32, vp, vp]
        L.trk_dipole_histogram.argtypes = [C.POINTER(BeamStruct), i32, vp, vp, vp, vp, sz, vp]
        L.trk_trwake_convolve.argtypes = [vp, i32, vp, d, d, i32, vp, vp]
        L.trk_trwake_kick.argtypes = [C.POINTER(BeamStruct), vp, i32, vp, C.POINTER(Wake), d,
                                      i32, vp, sz, vp]
        L.trk_wake_kick.argtypes = [C.POINTER(BeamStruct), vp, i32, vp, C.POINTER(Wake), d, i32,
                                    vp, sz, vp]
        L.trk_moments.argtypes = [C.POINTER(BeamStruct), vp, vp, sz, vp]
        L.trk_moments_noalloc.argtypes = [C.POINTER(BeamStruct), vp, vp]
        L.trk_moments_compensated.argtypes = [C.POINTER(BeamStruct), vp, vp, sz, vp]
        L.trk_compact_lost.argtypes = [C.POINTER(BeamStruct), vp, sz, vp]
        L.trk_compact_lost_mode.argtypes = [C.POINTER(BeamStruct), i32, vp, sz, vp]
        L.trk_elementary.argtypes = [i32, vp, vp, vp, i64, vp]
        L.trk_philox4x32_10.argtypes = [vp, vp, vp, i64, vp]
        L.trk_gauss.argtypes = [vp, u32, u32, u64, vp, i64, vp]
        L.trk_probe_stream.argtypes = [vp, vp, i64, i32, i32, vp]
        L.trk_probe_fma.argtypes = [vp, i32, i32, vp]
        L.trk_status_string.argtypes = [C.c_int]
        L.trk_status_string.restype = C.c_char_p
        L.trk_last_error.restype = C.c_char_p
        L.trk_profile_enable.argtypes = [i32]
        L.trk_profile_read.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.trk_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(i64), C.POINTER(u64),
                                       C.POINTER(vp)]
        L.trk_batch_destroy.argtypes = [vp]
        L.trk_batch_destroy.restype = None
        L.trk_batch_workspace_size.argtypes = [vp, i32]
        L.trk_batch_workspace_size.restype = sz
        L.trk_track_batched.argtypes = [vp, C.POINTER(BeamStruct), i32, i32,
                                        C.POINTER(BatchTuning), vp, vp, sz, vp]
        L.trk_mlp_create.argtypes = [vp, C.POINTER(vp)]
        L.trk_mlp_destroy.argtypes = [vp]
        L.trk_mlp_destroy.restype = None
        L.trk_mlp_get_params.argtypes = [vp, vp, vp]
        L.trk_mlp_forward.argtypes = [vp, vp, i64, vp, i32, vp]
        L.trk_mlp_workspace_size.argtypes = [i32]
        L.trk_mlp_workspace_size.restype = sz
        L.trk_mlp_backward.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, sz, vp]
        L.trk_mlp_adam_step.argtypes = [vp, vp, d, vp]
        L.trk_mlp_train.argtypes = [vp, vp, vp, i64, C.POINTER(C.c_double), C.POINTER(TrainOpts),
                                    vp, vp, sz, vp]
        L.trk_surrogate_create.argtypes = [vp, C.POINTER(SurrOpts), vp, C.POINTER(vp)]
        L.trk_surrogate_destroy.argtypes = [vp]
        L.trk_surrogate_destroy.restype = None
        L.trk_surrogate_get_info.argtypes = [vp, C.POINTER(SurrInfo)]
        L.trk_surrogate_workspace_size.argtypes = [vp, i64]
        L.trk_surrogate_workspace_size.restype = sz
        L.trk_surrogate_gate.argtypes = [vp, C.POINTER(BeamStruct), vp, vp]
        L.trk_surrogate_sample.argtypes = [vp, u64, u64, C.POINTER(BeamStruct), C.POINTER(u64),
                                           vp, sz, vp]
        L.trk_surrogate_pairs.argtypes = [vp, C.POINTER(BeamStruct), vp, vp, vp, vp, sz, vp]
        L.trk_surrogate_fit_scale.argtypes = [vp, vp, i64, vp, sz, vp]
        L.trk_surrogate_apply.argtypes = [vp, vp, C.POINTER(BeamStruct), i32, i32, vp, vp, sz, vp]
        _LIB = L
    return _LIB


def _check(status: int) -> None:
    if status != TRK_OK:
        raise TrkError(status, lib().trk_last_error().decode())


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t) -> int:
    return t.data_ptr()


# ------------------------------------------------------------------ lattice
class Lattice:
    """Device copy of a lattice (a list of inputs.Element descriptions)."""

    def __init__(self, elements):
        self.elements = list(elements)
        arr = (Element * max(1, len(self.elements)))()
        keep = []
        for i, e in enumerate(self.elements):
            r = arr[i]
            r.kind = KIND[e.kind]
            r.aperture = APER[e.aperture]
            r.order, r.nsteps, r.nbins = e.order, e.nsteps, e.nbins
            r.L, r.k, r.angle = e.L, e.k, e.angle
            r.volt, r.phase, r.freq = e.volt, e.phase, e.freq
            r.wake_A, r.wake_tau0, r.wake_omega, r.charge = (e.wake_A, e.wake_tau0,
                                                             e.wake_omega, e.charge)
            r.sigma, r.ax, r.ay = e.sigma, e.ax, e.ay
            if e.coef is not None:
                c = np.ascontiguousarray(e.coef, dtype=np.float64)
                need = {"MAP2": 168, "MAP3": 504}.get(e.kind)
                if need is not None and c.size != need:
                    raise ValueError(f"{e.kind} needs {need} coefficients, got {c.size}")
                keep.append(c)
                r.coef = c.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        _check(lib().trk_lattice_create(arr, len(self.elements), C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.trk_lattice_destroy(h)
            self.handle = None


# ------------------------------------------------------------------ beam
class Beam:
    """Device beam held in torch tensors: z [6, n] float64 (rows are the SoA
    coordinate arrays), id uint32 (as int32 storage), lost_at int64, n_alive."""

    def __init__(self, z, pid, lost_at, n_alive: Optional[int] = None, device="cuda"):
        import torch
        z = torch.as_tensor(np.ascontiguousarray(z), dtype=torch.float64)
        self.n = int(z.shape[1])
        self.z = z.to(device).contiguous()
        pid = np.ascontiguousarray(pid, dtype=np.uint32).view(np.int32)
        self.id = torch.as_tensor(pid).to(device).contiguous()
        self.lost_at = torch.as_tensor(np.ascontiguousarray(lost_at, dtype=np.int64)).to(device)
        na = self.n if n_alive is None else int(n_alive)
        self.n_alive = torch.tensor([na], dtype=torch.int64, device=device)
        self._struct = None

    @classmethod
    def from_inputs(cls, d: dict, device="cuda") -> "Beam":
        return cls(d["z"], d["id"], d["lost_at"], device=device)

    @classmethod
    def empty(cls, n: int, device="cuda") -> "Beam":
        """Device beam of n zeroed slots (ids 0..n-1, all alive), allocated on
        the device without a host copy."""
        import torch
        b = cls.__new__(cls)
        b.n = int(n)
        b.z = torch.zeros((6, b.n), dtype=torch.float64, device=device)
        b.id = torch.arange(b.n, dtype=torch.int64, device=device).to(torch.int32)
        b.lost_at = torch.full((b.n,), -1, dtype=torch.int64, device=device)
        b.n_alive = torch.tensor([b.n], dtype=torch.int64, device=device)
        b._struct = None
        return b

    def clone(self) -> "Beam":
        b = Beam.__new__(Beam)
        b.n = self.n
        b.z = self.z.clone()
        b.id = self.id.clone()
        b.lost_at = self.lost_at.clone()
        b.n_alive = self.n_alive.clone()
        b._struct = None
        return b

    def copy_(self, other: "Beam") -> None:
        self.z.copy_(other.z)
        self.id.copy_(other.id)
        self.lost_at.copy_(other.lost_at)
        self.n_alive.copy_(other.n_alive)

    def struct(self) -> BeamStruct:
        b = BeamStruct()
        zp = [self.z[k].data_ptr() for k in range(6)]
        b.x, b.xp, b.y, b.yp, b.s, b.dp = zp
        b.id = _ptr(self.id)
        b.lost_at = _ptr(self.lost_at)
        b.n_alive = _ptr(self.n_alive)
        b.n_total = self.n
        self._struct = b
        return b

    def host(self) -> dict:
        """Copy back (synchronises): z, id (uint32), lost_at, n_alive."""
        return {"z": self.z.cpu().numpy(), "id": self.id.cpu().numpy().view(np.uint32),
                "lost_at": self.lost_at.cpu().numpy(), "n_alive": int(self.n_alive.item())}


class Workspace:
    def __init__(self, n_total: int, lattice: Optional[Lattice] = None, device="cuda"):
        import torch
        nbytes = int(lib().trk_workspace_size(lattice.handle if lattice else None, n_total))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


# ------------------------------------------------------------------ calls
def track(beam: Beam, lattice: Lattice, passes: int, ws: Workspace, seed: int = 0,
          first_pass: int = 0, p_ref: float = 1e9, moments=None, wake_mode: int = WAKE_FP64,
          passes_per_launch: int = 0, max_elems_per_launch: int = 0, run_ppt: int = 0,
          run_blocks: int = 0, run_longit: int = 0, run_nt: int = 0, run_hist: int = 0,
          stream=None) -> None:
    o = Opts()
    o.run_ppt = run_ppt
    o.run_blocks = run_blocks
    o.run_longit = run_longit
    o.run_nt = run_nt
    o.run_hist = run_hist
    o.seed = seed
    o.first_pass = first_pass
    o.passes_per_launch = passes_per_launch
    o.max_elems_per_launch = max_elems_per_launch
    o.wake_mode = wake_mode
    o.p_ref_eV = p_ref
    o.moments = moments.data_ptr() if moments is not None else None
    _check(lib().trk_track(C.byref(beam.struct()), lattice.handle, passes, C.byref(o), ws.ptr,
                           ws.nbytes, _stream_handle(stream)))


def histogram(beam: Beam, nbins: int, ws: Workspace, stream=None):
    import torch
    rng = torch.empty(2, dtype=torch.float64, device=beam.z.device)
    cnt = torch.empty(nbins, dtype=torch.int32, device=beam.z.device)
    _check(lib().trk_histogram(C.byref(beam.struct()), nbins, rng.data_ptr(), cnt.data_ptr(),
                               ws.ptr, ws.nbytes, _stream_handle(stream)))
    return rng, cnt


def wake_convolve(counts, nbins: int, rng, tau0: float, omega: float, mode: int, stream=None):
    import torch
    v = torch.empty(nbins, dtype=torch.float64, device=rng.device)
    _check(lib().trk_wake_convolve(counts.data_ptr(), nbins, rng.data_ptr(), tau0, omega, mode,
                                   v.data_ptr(), _stream_handle(stream)))
    return v


def wake_kick(beam: Beam, counts, nbins: int, rng, A: float, tau0: float, omega: float,
              charge: float, p_ref: float, mode: int, ws: Workspace, stream=None) -> None:
    w = Wake(A, tau0, omega, charge)
    _check(lib().trk_wake_kick(C.byref(beam.struct()), counts.data_ptr(), nbins, rng.data_ptr(),
                               C.byref(w), p_ref, mode, ws.ptr, ws.nbytes, _stream_handle(stream)))


def dipole_histogram(beam: Beam, nbins: int, ws: Workspace, stream=None):
    """(range[2], counts[nbins], dipole[2][nbins] int64 in units of 2^-40 m)."""
    import torch
    dev = beam.z.device
    rng = torch.empty(2, dtype=torch.float64, device=dev)
    cnt = torch.empty(nbins, dtype=torch.int32, device=dev)
    dip = torch.empty((2, nbins), dtype=torch.int64, device=dev)
    _check(lib().trk_dipole_histogram(C.byref(beam.struct()), nbins, rng.data_ptr(),
                                      cnt.data_ptr(), dip.data_ptr(), ws.ptr, ws.nbytes,
                                      _stream_handle(stream)))
    return rng, cnt, dip


def trwake_convolve(dip, nbins: int, rng, tau0: float, omega: float, mode: int, stream=None):
    import torch
    v = torch.empty((2, nbins), dtype=torch.float64, device=rng.device)
    _check(lib().trk_trwake_convolve(dip.data_ptr(), nbins, rng.data_ptr(), tau0, omega, mode,
                                     v.data_ptr(), _stream_handle(stream)))
    return v


def trwake_kick(beam: Beam, dip, nbins: int, rng, A: float, tau0: float, omega: float,
                charge: float, p_ref: float, mode: int, ws: Workspace, stream=None) -> None:
    w = Wake(A, tau0, omega, charge)
    _check(lib().trk_trwake_kick(C.byref(beam.struct()), dip.data_ptr(), nbins, rng.data_ptr(),
                                 C.byref(w), p_ref, mode, ws.ptr, ws.nbytes,
                                 _stream_handle(stream)))


def moments(beam: Beam, ws: Workspace, stream=None):
    import torch
    out = torch.empty(28, dtype=torch.float64, device=beam.z.device)
    _check(lib().trk_moments(C.byref(beam.struct()), out.data_ptr(), ws.ptr, ws.nbytes,
                             _stream_handle(stream)))
    return out


def moments_compensated(beam: Beam, ws: Workspace, stream=None):
    """trk_moments_compensated: the moments with Kahan-compensated sums."""
    import torch
    out = torch.empty(28, dtype=torch.float64, device=beam.z.device)
    _check(lib().trk_moments_compensated(C.byref(beam.struct()), out.data_ptr(), ws.ptr,
                                         ws.nbytes, _stream_handle(stream)))
    return out


def moments_noalloc(beam: Beam, out, stream=None):
    """trk_moments_noalloc into the caller's device tensor out[28] (float64):
    no workspace, the library's static scratch."""
    _check(lib().trk_moments_noalloc(C.byref(beam.struct()), out.data_ptr(),
                                     _stream_handle(stream)))
    return out


COMPACT_STABLE, COMPACT_SWAP, COMPACT_SORT = 0, 1, 2


def compact_lost(beam: Beam, ws: Workspace, stream=None, mode: int = COMPACT_STABLE) -> None:
    if mode == COMPACT_STABLE:
        _check(lib().trk_compact_lost(C.byref(beam.struct()), ws.ptr, ws.nbytes,
                                      _stream_handle(stream)))
    else:
        _check(lib().trk_compact_lost_mode(C.byref(beam.struct()), mode, ws.ptr, ws.nbytes,
                                           _stream_handle(stream)))


def elementary(fn: int, x, y=None, stream=None):
    import torch
    out = torch.empty_like(x)
    _check(lib().trk_elementary(fn, x.data_ptr(), y.data_ptr() if y is not None else None,
                                out.data_ptr(), x.numel(), _stream_handle(stream)))
    return out


def philox(ctr, key, stream=None):
    import torch
    n = ctr.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    _check(lib().trk_philox4x32_10(ctr.data_ptr(), key.data_ptr(), out.data_ptr(), n,
                                   _stream_handle(stream)))
    return out


def gauss(pid, step: int, tag: int, seed: int, stream=None):
    import torch
    out = torch.empty(pid.shape[0], dtype=torch.float64, device=pid.device)
    _check(lib().trk_gauss(pid.data_ptr(), step, tag, seed, out.data_ptr(), pid.shape[0],
                           _stream_handle(stream)))
    return out


def probe_stream(src, dst, mode: int, blocks: int, stream=None) -> None:
    """mode 0: dst = src + 1 (dst as long as src); mode 1: dst[:blocks] =
    per-workgroup sums of src; mode 2: as 0 with non-temporal accesses."""
    _check(lib().trk_probe_stream(src.data_ptr(), dst.data_ptr(), src.numel(), mode, blocks,
                                  _stream_handle(stream)))


def probe_fma(out, iters: int, blocks: int, stream=None) -> None:
    """out[blocks * 256] doubles; 16 * iters flops per lane."""
    _check(lib().trk_probe_fma(out.data_ptr(), iters, blocks, _stream_handle(stream)))


def profile_enable(on, classes: int = 1) -> None:
    """Time launches with HIP events: `classes` is a bit mask (bit 0 fused
    runs, 1 surrogate inference, 2 wake histogram, 3 wake convolution)."""
    _check(lib().trk_profile_enable(int(classes) if on else 0))


def profile_read(cls: int = 0):
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().trk_profile_read(cls, C.byref(ms), C.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------------ batches
class Batch:
    """Variants of one lattice structure over a concatenated beam."""

    def __init__(self, lattices, seg_off, seeds):
        self.lattices = list(lattices)          # keep the handles alive
        nvar = len(self.lattices)
        hs = (C.c_void_p * nvar)(*[L.handle.value for L in self.lattices])
        off = np.ascontiguousarray(seg_off, dtype=np.int64)
        sd = np.ascontiguousarray(seeds, dtype=np.uint64)
        assert off.shape == (nvar + 1,) and sd.shape == (nvar,)
        h = C.c_void_p()
        _check(lib().trk_batch_create(hs, nvar, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                      sd.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(h)))
        self.handle = h
        self.nvar = nvar
        self.seg_off = off

    def workspace(self, passes_per_launch: int = 64, device="cuda"):
        import torch
        n = int(lib().trk_batch_workspace_size(self.handle, passes_per_launch))
        buf = torch.empty(n, dtype=torch.uint8, device=device)
        return buf

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.trk_batch_destroy(h)
            self.handle = None


def track_batched(batch: Batch, beam: Beam, passes: int, ws, first_pass: int = 0, ppt: int = 1,
                  blocks_per_cu: int = 2, passes_per_launch: int = 0, use_graph: bool = True,
                  moments=None, stream=None) -> None:
    t = BatchTuning(ppt, blocks_per_cu, passes_per_launch, 1 if use_graph else 0)
    _check(lib().trk_track_batched(batch.handle, C.byref(beam.struct()), passes, first_pass,
                                   C.byref(t), moments.data_ptr() if moments is not None else None,
                                   ws.data_ptr(), ws.numel(), _stream_handle(stream)))


# ------------------------------------------------------------------ surrogate
class Mlp:
    """Device copy of the residual network (FP32 master weights, Adam state,
    bfloat16 copies)."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (MLP_NPARAM,)
        h = C.c_void_p()
        _check(lib().trk_mlp_create(p.ctypes.data, C.byref(h)))
        self.handle = h

    def params(self, stream=None) -> np.ndarray:
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        _check(lib().trk_mlp_get_params(self.handle, out.ctypes.data, _stream_handle(stream)))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.trk_mlp_destroy(h)
            self.handle = None


def mlp_forward(m: Mlp, u, precision: int = MLP_BF16X2, stream=None):
    """u: device float32 [n, 8] -> device float32 [n, 8]"""
    import torch
    out = torch.empty_like(u)
    _check(lib().trk_mlp_forward(m.handle, u.data_ptr(), int(u.shape[0]), out.data_ptr(),
                                 precision, _stream_handle(stream)))
    return out


def mlp_workspace(batch: int, device="cuda"):
    import torch
    return torch.empty(int(lib().trk_mlp_workspace_size(batch)), dtype=torch.uint8, device=device)


def mlp_backward(m: Mlp, u, t, ws, precision: int = MLP_BF16X2, stream=None):
    """Gradient (device float32 [NPARAM]) and loss (device float32 [1])."""
    import torch
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=u.device)
    loss = torch.empty(1, dtype=torch.float32, device=u.device)
    _check(lib().trk_mlp_backward(m.handle, u.data_ptr(), t.data_ptr(), int(u.shape[0]), precision,
                                  g.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream_handle(stream)))
    return g, loss


def mlp_adam_step(m: Mlp, grad, lr: float, stream=None) -> None:
    _check(lib().trk_mlp_adam_step(m.handle, grad.data_ptr(), lr, _stream_handle(stream)))


def mlp_train(m: Mlp, u, r, inv_scale, ws, batch: int, epochs: int, lr0: float, lr_min: float,
              seed: int = 0, precision: int = MLP_BF16X2, n_pairs: Optional[int] = None,
              stream=None):
    """Returns the per-epoch mean batch loss (device float32 [epochs])."""
    import torch
    o = TrainOpts(batch, epochs, precision, 0, lr0, lr_min, seed)
    sc = (C.c_double * 6)(*[float(v) for v in inv_scale])
    loss = torch.zeros(max(epochs, 1), dtype=torch.float32, device=u.device)
    n = int(u.shape[0]) if n_pairs is None else int(n_pairs)
    _check(lib().trk_mlp_train(m.handle, u.data_ptr(), r.data_ptr(), n, sc, C.byref(o),
                               loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return loss


class Surrogate:
    """Section handle: linear map, gate constants, residual scale."""

    def __init__(self, section: Lattice, half_width, margin: float, aper=(10e-3, 5e-3),
                 h_rel: float = 1e-4, stream=None):
        o = SurrOpts()
        for k in range(6):
            o.half_width[k] = float(half_width[k])
        o.margin, o.h_rel = float(margin), float(h_rel)
        o.aper_a, o.aper_b = float(aper[0]), float(aper[1])
        h = C.c_void_p()
        _check(lib().trk_surrogate_create(section.handle, C.byref(o), _stream_handle(stream),
                                          C.byref(h)))
        self.handle = h
        self.section = section                  # keep the lattice alive

    def info(self) -> dict:
        i = SurrInfo()
        _check(lib().trk_surrogate_get_info(self.handle, C.byref(i)))
        out = {k: getattr(i, k) for k, _ in SurrInfo._fields_}
        out["C"] = np.array(list(i.C))
        out["R"] = np.array(list(i.R)).reshape(6, 6)
        out["D"] = np.array(list(i.D))
        out["sample_half_width"] = np.array(list(i.sample_half_width))
        return out

    def workspace(self, n_total: int, device="cuda"):
        import torch
        nb = int(lib().trk_surrogate_workspace_size(self.handle, n_total))
        return torch.empty(nb, dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.trk_surrogate_destroy(h)
            self.handle = None


def surrogate_gate(s: Surrogate, beam: Beam, stream=None):
    import torch
    adm = torch.zeros(max(beam.n, 1), dtype=torch.uint8, device=beam.z.device)
    _check(lib().trk_surrogate_gate(s.handle, C.byref(beam.struct()), adm.data_ptr(),
                                    _stream_handle(stream)))
    return adm[:beam.n]


def surrogate_sample(s: Surrogate, seed: int, first: int, beam: Beam, ws, stream=None) -> int:
    nxt = C.c_uint64()
    _check(lib().trk_surrogate_sample(s.handle, seed, first, C.byref(beam.struct()), C.byref(nxt),
                                      ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return int(nxt.value)


def surrogate_pairs(s: Surrogate, beam: Beam, ws, stream=None):
    """(u [n, 8], r [n, 8], n_pairs device int64 [1]) for the beam's admitted particles."""
    import torch
    u = torch.zeros((max(beam.n, 1), 8), dtype=torch.float32, device=beam.z.device)
    r = torch.zeros_like(u)
    n = torch.zeros(1, dtype=torch.int64, device=beam.z.device)
    _check(lib().trk_surrogate_pairs(s.handle, C.byref(beam.struct()), u.data_ptr(), r.data_ptr(),
                                     n.data_ptr(), ws.data_ptr(), ws.numel(),
                                     _stream_handle(stream)))
    return u, r, n


def surrogate_fit_scale(s: Surrogate, r, n: int, ws, stream=None) -> np.ndarray:
    _check(lib().trk_surrogate_fit_scale(s.handle, r.data_ptr(), int(n), ws.data_ptr(), ws.numel(),
                                         _stream_handle(stream)))
    return s.info()["D"]


def surrogate_apply(s: Surrogate, m: Mlp, beam: Beam, ws, first_pass: int = 0,
                    precision: int = MLP_BF16X2, n_admitted=None, stream=None) -> None:
    _check(lib().trk_surrogate_apply(s.handle, m.handle, C.byref(beam.struct()), first_pass,
                                     precision,
                                     n_admitted.data_ptr() if n_admitted is not None else None,
                                     ws.data_ptr(), ws.numel(), _stream_handle(stream)))

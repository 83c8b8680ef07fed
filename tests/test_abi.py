"""The C-ABI library loads on a host without a GPU and exports every function
that include/trk.h declares (no compute calls here)."""
import os
import re
import subprocess

from paper_1710_07350_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "trk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trk_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_set():
    assert declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    nm = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(trk_\w+)", nm))
    for name in declared():
        assert name in exported, name
        assert hasattr(lib, name), name


def test_status_strings_and_sizes():
    lib = binding.lib()
    assert lib.trk_status_string(0) == b"ok"
    assert lib.trk_status_string(binding.TRK_EPTR).startswith(b"host pointer")
    # workspace grows with the beam and is at least the staging copy (60 B/particle)
    small = lib.trk_workspace_size(None, 1000)
    big = lib.trk_workspace_size(None, 1_000_000)
    assert big > small and big >= 60 * 1_000_000


def test_invalid_lattice_rejected_without_gpu():
    from paper_1710_07350_amd.inputs import Element
    import pytest
    with pytest.raises(binding.TrkError) as e:
        binding.Lattice([Element("WAKE", nbins=1, wake_tau0=1e-11)])
    assert e.value.status == binding.TRK_EINVAL
    with pytest.raises(binding.TrkError):
        binding.Lattice([Element("MULT", k=1.0, order=0)])


def test_surrogate_host_checks_without_gpu():
    import ctypes as C
    lib = binding.lib()
    # sizes are pure host arithmetic
    assert lib.trk_mlp_workspace_size(0) == 0
    w1, w2 = lib.trk_mlp_workspace_size(64), lib.trk_mlp_workspace_size(8192)
    assert 0 < w1 < w2
    s1 = lib.trk_surrogate_workspace_size(None, 1000)
    s2 = lib.trk_surrogate_workspace_size(None, 10_000_000)
    assert 0 < s1 < s2 and s2 >= 100 * 10_000_000
    # NULL handles and bad arguments are rejected before any device call
    h = C.c_void_p()
    assert lib.trk_mlp_create(None, C.byref(h)) == binding.TRK_EINVAL
    assert lib.trk_surrogate_create(None, None, None, C.byref(h)) == binding.TRK_EINVAL
    assert lib.trk_mlp_forward(None, None, 0, None, 0, None) == binding.TRK_EINVAL
    o = binding.TrainOpts(64, 1, 0, 0, 1e-3, 1e-5, 0)
    sc = (C.c_double * 6)(*([1.0] * 6))
    assert lib.trk_mlp_train(None, None, None, 64, sc, C.byref(o), None, None, 0,
                             None) == binding.TRK_EINVAL
    info = binding.SurrInfo()
    assert lib.trk_surrogate_get_info(None, C.byref(info)) == binding.TRK_EINVAL


def test_transverse_wake_host_checks_without_gpu():
    from paper_1710_07350_amd.inputs import Element
    import pytest
    lib = binding.lib()
    for nb in (1, 2049):
        with pytest.raises(binding.TrkError) as e:
            binding.Lattice([Element("TRWAKE", nbins=nb, wake_tau0=1e-11)])
        assert e.value.status == binding.TRK_EINVAL
    with pytest.raises(binding.TrkError):
        binding.Lattice([Element("TRWAKE", nbins=64, wake_tau0=0.0)])
    # bin counts beyond the transverse limit are rejected before any device call
    assert lib.trk_dipole_histogram(None, 4096, None, None, None, None, 0, None) == \
        binding.TRK_ERANGE
    assert lib.trk_trwake_convolve(None, 1, None, 1e-11, 0.0, 0, None, None) == binding.TRK_ERANGE
    assert lib.trk_trwake_convolve(None, 64, None, 1e-11, 0.0, 7, None, None) == binding.TRK_EINVAL


def test_compaction_mode_checked_without_gpu():
    lib = binding.lib()
    assert lib.trk_compact_lost_mode(None, 9, None, 0, None) == binding.TRK_EINVAL

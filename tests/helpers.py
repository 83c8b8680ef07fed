"""Shared helpers of the GPU parity tests: run the same seeded input through
the HIP library (via its C-ABI binding) and through the CPU oracle."""
import numpy as np

import oracle
from paper_1710_07350_amd import binding as B

COORD_SCALE = np.array([1e-3, 1e-4, 1e-3, 1e-4, 1e-3, 1e-3])


def rel_err(a, b, scale=COORD_SCALE):
    """Per-coordinate error |a-b| / max(|b|, sigma_k), the parity metric that
    avoids spurious relative errors of coordinates near zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.maximum(np.abs(b), scale[:, None])
    with np.errstate(invalid="ignore"):
        e = np.abs(a - b) / den
    both_nan = np.isnan(a) & np.isnan(b)
    e[both_nan] = 0.0
    return float(np.nanmax(e)) if e.size else 0.0


def run_gpu(lat, d, passes, p_ref=1e9, seed=0, moments=False, n_alive=None, **kw):
    import torch
    beam = B.Beam.from_inputs(d)
    if n_alive is not None:
        beam.n_alive.fill_(n_alive)
    ws = B.Workspace(beam.n)
    L = B.Lattice(lat)
    mom = torch.zeros((max(passes, 1), 28), dtype=torch.float64, device="cuda") if moments else None
    B.track(beam, L, passes, ws, seed=seed, p_ref=p_ref, moments=mom, **kw)
    torch.cuda.synchronize()
    out = beam.host()
    out["moments"] = mom.cpu().numpy() if moments else None
    return out


def run_oracle(lat, d, passes, p_ref=1e9, seed=0, moments=False, first_pass=0):
    b = oracle.Beam.from_inputs(d)
    n, mom = oracle.track(b, lat, passes, first_pass=first_pass, p_ref=p_ref, seed=seed,
                          moments=moments)
    return {"z": b.z, "id": b.id, "lost_at": b.lost_at, "n_alive": n, "moments": mom}


def assert_bit_exact(g, r):
    assert g["n_alive"] == r["n_alive"], (g["n_alive"], r["n_alive"])
    assert np.array_equal(g["id"], r["id"])
    assert np.array_equal(g["lost_at"], r["lost_at"])
    err = rel_err(g["z"], r["z"])
    assert err <= 1e-12, err
    same = (g["z"] == r["z"]) | (np.isnan(g["z"]) & np.isnan(r["z"]))
    assert same.all(), f"{(~same).sum()} coordinates differ (max rel err {err:.3e})"


def moments_close(gm, rm, rtol=1e-12):
    """Moment rows agree: n exactly, means and second moments relative to the
    beam's scale (sigma_k for means, sigma_k sigma_l for second moments)."""
    gm = np.atleast_2d(gm)
    rm = np.atleast_2d(rm)
    assert np.array_equal(gm[:, 0], rm[:, 0])
    sig = np.sqrt(np.maximum(np.abs(rm[:, 7 + np.array([0, 6, 11, 15, 18, 20])]), 1e-300))
    for p in range(rm.shape[0]):
        for k in range(6):
            assert abs(gm[p, 1 + k] - rm[p, 1 + k]) <= rtol * max(sig[p, k], abs(rm[p, 1 + k]))
        o = 7
        for k in range(6):
            for l in range(k, 6):
                assert abs(gm[p, o] - rm[p, o]) <= rtol * sig[p, k] * sig[p, l], (p, k, l)
                o += 1

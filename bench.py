#!/usr/bin/env python3
"""Throughput benchmark: particle-element steps per second on one MI355X.

Default workload: the linac bunch compressor -- 4e6 particles of a chirped 6D
Gaussian beam through 8 zero-length RF cavities, each followed by the
longitudinal wake step (1024-bin histogram of s, FP32 matrix-core causal
convolution with a resonator wake, interpolated energy kick), then a
second-order chicane map (17 elements per pass).  One step = one pass of a
fresh, already device-resident batch.  A particle-element step is one element
applied to one particle alive at its entry.

Prints one JSON line with the throughput, the roofline position of the
dominant kernel (the fused element-run kernel, timed with HIP events on its
stream during the timed steps) and the CPU oracle timed on a bounded sample.

  python bench.py [--steps K] [--warmup W] [--workload bc|ring|fodo|roof|surr]

The surr workload measures the learned section surrogate instead: it trains
the network on the GPU (pairs from the tracker over the admitted part of the
+-6 sigma box), then times one pass through the first ten ring cells with
plain tracking and with gate + network + fallback on 1e7 fresh particles,
and reports the speed-up and the surrogate's error against the tracker.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WAKES = ("WAKE", "TRWAKE")
# HBM bytes of the dominant kernel per launch, keyed by (workload, element
# limit per launch), from rocprofv3 FETCH_SIZE and WRITE_SIZE (FETCH_SIZE
# scaled by 2.000, WRITE_SIZE by 1.000, the factors a 1 GiB copy gives),
# averaged over the runs of one pass (profiles/*_hbm_bytes.md); absent until
# measured for the current kernel.
TRAFFIC_PER_LAUNCH = {("bc", 0): 101947278, ("roof", 1): 734090445}
# FP64 vector peak (dense, FMA = 2 flops) and the FP64 flops of one
# particle-element step of each lattice: SQ_INSTS_VALU_FLOPS_FP64 (2 FMA + MUL
# + ADD + TRANS per wave instruction) x 64 lanes over the exact steps of a
# run in which nobody is lost (profiles/k_run_fp64_flops.md)
FP64_PEAK_TFLOPS = 78.6
FP64_FLOP_PER_STEP = {"ring": 135.8, "fodo": 60.0, "fodo3": 72.7}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="bc",
                    choices=["bc", "rfcw", "ring", "fodo", "roof", "surr", "batch", "compact"])
    ap.add_argument("--epochs", type=int, default=20, help="surrogate training epochs")
    ap.add_argument("--precision", default="bf16x2", choices=["bf16", "bf16x2"])
    ap.add_argument("--wake-mode", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--fusion", type=int, default=0, help="max elements per launch (roof)")
    ap.add_argument("--quad-order", type=int, default=2, choices=[2, 3],
                    help="fodo/roof: track the quadrupoles with second- or third-order maps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--particles", type=float, default=None)
    ap.add_argument("--sigma-scale", type=float, default=1.0,
                    help="scale the Gaussian beam's sigmas (0.1: nobody is lost)")
    return ap.parse_args()


def run_mask_bytes(lattice, e0, e1, moments=False, next_wake=False):
    """Algorithmic bytes per particle of one fused launch over elements
    [e0, e1): each coordinate read by the run is loaded once and each one it
    changes is stored once (8 B each), the id (4 B) when a random kick needs
    it, and the 8-byte loss record of particles lost in the run (not counted:
    data dependent and small)."""
    rd, wr, need_id = set(), set(), False
    for e in lattice[e0:e1]:
        k = e.kind
        if k == "EDRIFT":
            rd |= {0, 1, 2, 3, 4}; wr |= {0, 2, 4}
        elif k in ("QUAD", "MAP2", "MAP3"):
            c = e.coef if e.coef is not None else None
            if k == "MAP2":
                R = c[6:42].reshape(6, 6); T = c[42:].reshape(6, 21)
                for i in range(6):
                    ident = c[i] == 0 and R[i, i] == 1 and np.count_nonzero(R[i]) == 1 \
                        and not T[i].any()
                    if ident:
                        continue
                    wr.add(i)
                    rd |= set(np.nonzero(R[i])[0].tolist())
                    pairs = [(j, kk) for j in range(6) for kk in range(j, 6)]
                    for q in np.nonzero(T[i])[0]:
                        rd |= set(pairs[q])
            else:
                rd |= set(range(6)); wr |= {0, 1, 2, 3, 4}
        elif k == "MULT":
            rd |= {0, 1, 2, 3, 5}; wr |= {1, 3}
        elif k in ("KQUAD", "CSBEND"):
            rd |= set(range(6)); wr |= {0, 1, 2, 3, 4}
        elif k in ("RFCA", "WAKE"):
            rd |= {4, 5}; wr |= {5}
        elif k == "TRWAKE":
            rd |= {1, 3, 4, 5}; wr |= {1, 3}
        elif k == "RADKICK":
            rd |= {5}; wr |= {5}; need_id = True
        if e.aperture != "NONE":
            rd |= {0, 2}
    if moments:
        rd |= set(range(6))
    if next_wake:
        rd |= {4}
    rd |= wr
    return 8 * len(rd) + 8 * len(wr) + (4 if need_id else 0)


def launches_of(lattice, passes_per_launch=16, max_e=0):
    """(e0, e1, npass) of each fused launch, as the library plans them."""
    n = len(lattice)
    has_wake = any(e.kind in WAKES for e in lattice)
    if not has_wake and (max_e == 0 or max_e >= n):
        return [(0, n, passes_per_launch)]
    out, e0 = [], 0
    lim = max_e if max_e > 0 else n
    while e0 < n:
        e1 = e0 + 1
        while e1 < n and lattice[e1].kind not in WAKES and e1 - e0 < lim:
            e1 += 1
        out.append((e0, e1, 1))
        e0 = e1
    return out


def cpu_baseline(lattice, beam_kw, passes, p_ref, sample_n, seed=0):
    import oracle
    from paper_1710_07350_amd import inputs
    d = inputs.gaussian_beam(sample_n, **{k: v for k, v in beam_kw.items() if k != "n"})
    b = oracle.Beam.from_inputs(d)
    t0 = time.perf_counter()
    oracle.track(b, lattice, passes, p_ref=p_ref, seed=seed)
    dt = time.perf_counter() - t0
    steps = element_steps(lattice, passes, sample_n, b.lost_at, 0)
    return steps / dt, dt, oracle.get_threads()


def element_steps(lattice, passes, n, lost_at, first_pass):
    """Exact particle-element steps: survivors traverse every element of every
    pass; a particle lost at (pass, element) traversed up to that element."""
    nel = len(lattice)
    la = np.asarray(lost_at)
    lost = la[la >= 0]
    alive = int((la < 0).sum())
    p = (lost >> 32) - first_pass
    e = lost & 0xFFFFFFFF
    return float(alive) * passes * nel + float((p * nel + e + 1).sum())


def surrogate_bench(args):
    """Train the section surrogate, then time plain tracking against
    gate + network + fallback on fresh particles of two distributions."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    torch.cuda.set_device(0)
    n = int(args.particles or 10_000_000)
    prec = B.MLP_BF16X2 if args.precision == "bf16x2" else B.MLP_BF16
    margin, aper = 0.5, (10e-3, 5e-3)
    hw = 6.0 * np.array(inputs.BEAM_SIGMAS)
    sec = inputs.ring_lattice(seed=0)[:100]
    L = B.Lattice(sec)
    sur = B.Surrogate(L, hw, margin, aper)
    ws = sur.workspace(n)
    # training pairs: n admitted inputs from the sampler, tracked through the section
    t0 = time.perf_counter()
    beam = B.Beam.empty(n)
    B.surrogate_sample(sur, 5, 0, beam, ws)
    u, r, npairs_t = B.surrogate_pairs(sur, beam, ws)
    npairs = int(npairs_t.item())
    D = B.surrogate_fit_scale(sur, r, npairs, ws)
    del beam
    t_pairs = time.perf_counter() - t0
    print(f"pairs: {npairs} in {t_pairs:.2f} s; D = {D}", file=sys.stderr, flush=True)
    inv = [1.0 / v if v > 0 else 0.0 for v in D]
    m = B.Mlp(inputs.mlp_init_params(21))
    batch = 8192
    mws = B.mlp_workspace(batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = B.mlp_train(m, u, r, inv, mws, batch=batch, epochs=args.epochs, lr0=2e-3,
                       lr_min=1e-5, seed=9, precision=prec, n_pairs=npairs).cpu().numpy()
    t_train = time.perf_counter() - t0
    print(f"training: {args.epochs} epochs in {t_train:.1f} s, loss {loss[0]:.3e} -> "
          f"{loss[-1]:.3e}", file=sys.stderr, flush=True)
    del u, r

    def one_set(d, name, reps=5):
        src = B.Beam.from_inputs(d)
        work = src.clone()
        tws = B.Workspace(n)
        times = {"plain": [], "surr": []}
        B.profile_enable(True, classes=0b10)
        for rep in range(reps + 1):
            for mode in ("plain", "surr"):
                work.copy_(src)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                if mode == "plain":
                    B.track(work, L, 1, tws)
                else:
                    B.surrogate_apply(sur, m, work, ws, precision=prec)
                b.record()
                torch.cuda.synchronize()
                if rep > 0:
                    times[mode].append(a.elapsed_time(b))
                if rep == reps:
                    if mode == "plain":
                        ref = work.host()
                    else:
                        got = work.host()
        infer_ms, infer_n = B.profile_read(1)
        B.profile_enable(False)
        # surrogate error on admitted particles against the tracker, by id
        nadm = torch.zeros(1, dtype=torch.int64, device="cuda")
        work.copy_(src)
        adm = B.surrogate_gate(sur, work).cpu().numpy().astype(bool)
        ids = d["id"][adm]
        pos_r = np.empty(n, np.int64)
        pos_r[ref["id"]] = np.arange(n)
        pos_g = np.empty(n, np.int64)
        pos_g[got["id"]] = np.arange(n)
        zr = ref["z"][:, pos_r[ids]]
        zg = got["z"][:, pos_g[ids]]
        lost_adm = int((ref["lost_at"][pos_r[ids]] >= 0).sum())
        err = np.abs(zg - zr)
        names = ["x", "xp", "y", "yp", "s", "dp"]
        tp = float(np.median(times["plain"]))
        ts = float(np.median(times["surr"]))
        steps = element_steps(sec, 1, n, ref["lost_at"], 0)
        out = {"set": name, "particles": n, "admitted": int(adm.sum()),
               "admitted_lost_in_tracking": lost_adm,
               "ms_plain": round(tp, 3), "ms_surrogate": round(ts, 3),
               "speedup": round(tp / ts, 3),
               "steps_per_s_plain": steps / (tp / 1e3),
               "max_abs_error": {k: float(err[i].max()) if err.size else 0.0
                                 for i, k in enumerate(names)},
               "rms_error": {k: float(np.sqrt((err[i] ** 2).mean())) if err.size else 0.0
                             for i, k in enumerate(names)},
               "infer_ms": infer_ms / max(infer_n, 1)}
        print(json.dumps(out), file=sys.stderr, flush=True)
        return out

    fresh = B.Beam.empty(n)
    B.surrogate_sample(sur, 63, 0, fresh, ws)
    fh = fresh.host()
    del fresh
    dom = one_set({"z": fh["z"], "id": fh["id"], "lost_at": fh["lost_at"]},
                  "fresh uniform points of the training domain (box ∩ gate)")
    box = one_set(inputs.uniform_box_beam(n, seed=61, half_widths=hw), "uniform +-6 sigma box")
    gauss = one_set(inputs.gaussian_beam(n, seed=62), "Gaussian ring beam")
    # 100 ring turns of 1e6 particles: the section served by the surrogate for
    # admitted particles each turn (the rest of the ring tracked plainly),
    # against the whole ring tracked plainly; Philox kicks are keyed by
    # (id, turn), so both runs see the same kicks.
    nr, turns = 1_000_000, 100
    ring = inputs.ring_lattice(seed=0)
    Lring, Lrest = B.Lattice(ring), B.Lattice(ring[100:])
    d0 = inputs.gaussian_beam(nr, seed=64)
    plain, served = B.Beam.from_inputs(d0), B.Beam.from_inputs(d0)
    wsr = B.Workspace(nr)
    wss = sur.workspace(nr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(turns):
        B.track(plain, Lring, 1, wsr, seed=7, first_pass=t)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    nadm = torch.zeros(1, dtype=torch.int64, device="cuda")
    adm_sum = 0
    t0 = time.perf_counter()
    for t in range(turns):
        B.surrogate_apply(sur, m, served, wss, first_pass=t, precision=prec, n_admitted=nadm)
        B.track(served, Lrest, 1, wsr, seed=7, first_pass=t)
        adm_sum += nadm
    torch.cuda.synchronize()
    t_served = time.perf_counter() - t0
    hp, hs = plain.host(), served.host()
    both = np.intersect1d(hp["id"][:hp["n_alive"]], hs["id"][:hs["n_alive"]])
    pp = np.empty(nr, np.int64)
    pp[hp["id"]] = np.arange(nr)
    ps = np.empty(nr, np.int64)
    ps[hs["id"]] = np.arange(nr)
    drift = np.abs(hs["z"][:, ps[both]] - hp["z"][:, pp[both]])
    ring100 = {"particles": nr, "turns": turns, "alive_plain": hp["n_alive"],
               "alive_served": hs["n_alive"],
               "admitted_per_turn": float(adm_sum.item()) / turns / nr,
               "s_plain": round(t_plain, 3), "s_served": round(t_served, 3),
               "max_drift": {k: float(drift[i].max()) for i, k in
                             enumerate(["x", "xp", "y", "yp", "s", "dp"])},
               "rms_drift": {k: float(np.sqrt((drift[i] ** 2).mean())) for i, k in
                             enumerate(["x", "xp", "y", "yp", "s", "dp"])}}
    print(json.dumps(ring100), file=sys.stderr, flush=True)
    flops = 2.0 * (6 * 256 + 2 * 256 * 256 + 256 * 6)
    ach = dom["admitted"] * flops / (dom["infer_ms"] / 1e3) / 1e12
    mx = dom["max_abs_error"]
    out = {"metric": "surrogate speedup over plain tracking of the section",
           "value": dom["speedup"], "unit": "x", "n_gpus": 1, "steps": 5, "warmup": 1,
           "ms_per_step": dom["ms_surrogate"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16 network (" + args.precision + " activations), "
                                              "f64 linear part and fallback",
           "data": "synthetic",
           "config": {"workload": "learned surrogate of ring cells 0-9 (100 elements), "
                                  f"1e7 fresh particles, gate margin {margin}",
                      "training_pairs": npairs, "epochs": args.epochs, "batch": batch,
                      "train_s": round(t_train, 2), "final_loss": float(loss[-1])},
           "error": {"max_m": max(mx["x"], mx["y"], mx["s"]), "max_rad": max(mx["xp"], mx["yp"]),
                     "meets_1e-6": max(mx.values()) <= 1e-6},
           "sets": [dom, box, gauss],
           "ring_100_turns": ring100,
           "roofline": {"bound": "mfma", "kernel": "trk::k_surr_infer", "achieved": round(ach, 2),
                        "peak": 2500.0, "unit": "TFLOP/s", "frac": round(ach / 2500.0, 4),
                        "traffic": None}}
    print(json.dumps(out))


def batch_bench(args):
    """256 ring variants (own sextupoles, own seeds, log-uniform sizes in
    [1e3, 1e5]) in one persistent launch sequence (autotuned, hipGraph),
    against the same variants tracked one at a time with trk_track."""
    import torch
    from paper_1710_07350_amd import autotune
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    torch.cuda.set_device(0)
    nvar = 256
    turns = args.steps or 20
    sizes = inputs.batch_variant_sizes(nvar, seed=0)
    lats = [inputs.ring_lattice(seed=100 + v) for v in range(nvar)]
    beams = [inputs.gaussian_beam(int(n), seed=1000 + v) for v, n in enumerate(sizes)]
    seeds = np.array([7 + 13 * v for v in range(nvar)], dtype=np.uint64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = {"z": np.concatenate([b["z"] for b in beams], axis=1),
           "id": np.concatenate([b["id"] for b in beams]),
           "lost_at": np.concatenate([b["lost_at"] for b in beams])}
    Ls = [B.Lattice(l) for l in lats]
    bt = B.Batch(Ls, seg, seeds)
    src = B.Beam.from_inputs(cat)
    work = src.clone()
    t0 = time.perf_counter()
    tune = autotune.tune_batch(bt, work, probe_passes=4)
    t_tune = time.perf_counter() - t0
    print(f"autotune: {tune} in {t_tune:.1f} s", file=sys.stderr, flush=True)
    tune = {k: tune[k] for k in ("ppt", "blocks_per_cu", "passes_per_launch")}
    ws = bt.workspace(64)
    mom = torch.zeros((nvar, turns, 28), dtype=torch.float64, device="cuda")

    def batched():
        work.copy_(src)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        B.track_batched(bt, work, turns, ws, moments=mom, use_graph=True, **tune)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    batched()                                   # capture the graph
    tb = float(np.median([batched() for _ in range(3)]))
    res_b = work.host()
    # one at a time
    vb = [B.Beam.from_inputs(b) for b in beams]
    vws = [B.Workspace(int(n)) for n in sizes]
    vmom = [torch.zeros((turns, 28), dtype=torch.float64, device="cuda") for _ in range(nvar)]
    init = [(b.z.clone(), b.id.clone(), b.lost_at.clone(), b.n_alive.clone()) for b in vb]

    def sequential():
        for b, (z, i, l, na) in zip(vb, init):
            b.z.copy_(z); b.id.copy_(i); b.lost_at.copy_(l); b.n_alive.copy_(na)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        for v in range(nvar):
            B.track(vb[v], Ls[v], turns, vws[v], seed=int(seeds[v]), moments=vmom[v])
        e.record()
        torch.cuda.synchronize()
        return a.elapsed_time(e)

    sequential()
    ts = float(np.median([sequential() for _ in range(3)]))
    # variant by variant: identical particles (by id) and loss records
    same = True
    for v in range(nvar):
        h = vb[v].host()
        sl = slice(seg[v], seg[v + 1])
        o1 = np.argsort(res_b["id"][sl], kind="stable")
        o2 = np.argsort(h["id"], kind="stable")
        same &= bool(np.array_equal(res_b["z"][:, sl][:, o1], h["z"][:, o2]) and
                     np.array_equal(res_b["lost_at"][sl][o1], h["lost_at"][o2]))
    steps = element_steps(lats[0], turns, int(seg[-1]), res_b["lost_at"], 0)
    out = {"metric": "particle\u00b7element steps/s (batched ring scan)",
           "value": steps / (tb / 1e3), "unit": "particle\u00b7element steps/s",
           "n_gpus": 1, "steps": turns, "warmup": 1, "ms_per_step": tb / turns,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"batched scan: {nvar} ring variants, {int(seg[-1])} particles "
                                  f"(log-uniform 1e3-1e5 per variant), {turns} turns, moments "
                                  "every turn", "tuning": tune, "autotune_s": round(t_tune, 2)},
           "sequential": {"value": steps / (ts / 1e3), "ms": ts},
           "batched_ms": tb, "speedup_vs_sequential": ts / tb,
           "variants_identical_to_sequential": same}
    # the batched launch is bound by FP64 arithmetic, as the ring's run kernel
    # (same elements): its FP64 flops per element step over the whole job
    fl = FP64_FLOP_PER_STEP["ring"] * steps
    ach = fl / (tb / 1e3) / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "trk::k_batch (persistent; whole batched call)",
                       "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": None,
                       "fp64_flops_per_element_step": FP64_FLOP_PER_STEP["ring"]}
    if not args.no_cpu_baseline:
        # the oracle on variant 0 (its own sextupoles, beam and key), all turns
        cv, cdt, cores = cpu_baseline(lats[0], dict(seed=1000), turns, 1e9, int(sizes[0]),
                                      seed=int(seeds[0]))
        out["cpu_baseline"] = {"value": cv, "unit": "particle\u00b7element steps/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"variant 0 ({int(sizes[0])} particles), {turns} turns, "
                                         f"{cdt:.1f} s wall"}
    print(json.dumps(out))


def compact_bench(args):
    """The paper's comparison of loss reorderings (Sec. 2.5): time the stable
    reordering, the paper's sparse swap and the sort by key on 4e6 particles
    with 0.5, 5, 10 and 50 % of them lost at random slots."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = int(args.particles or 4_000_000)
    reps = args.steps or 10
    d = inputs.gaussian_beam(n, seed=0)
    tmpl = B.Beam.from_inputs(d)
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(n)
    stream = torch.cuda.current_stream()
    modes = {"stable": B.COMPACT_STABLE, "swap": B.COMPACT_SWAP, "sort": B.COMPACT_SORT}
    rng = np.random.default_rng(1)
    rows = []
    for frac in (0.005, 0.05, 0.1, 0.5):
        la = np.full(n, -1, np.int64)
        sel = rng.random(n) < frac
        la[sel] = (rng.integers(0, 9, sel.sum()) << 32) | rng.integers(0, 401, sel.sum())
        lost_t = torch.tensor(la, device="cuda")
        for name, mode in modes.items():
            times = []
            for r in range(reps + 1):
                beam.z.copy_(tmpl.z)
                beam.id.copy_(tmpl.id)
                beam.lost_at.copy_(lost_t)
                beam.n_alive.fill_(n)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.compact_lost(beam, ws, stream=stream, mode=mode)
                e1.record(stream)
                torch.cuda.synchronize()
                if r > 0:
                    times.append(e0.elapsed_time(e1))
            assert int(beam.n_alive.item()) == n - int(sel.sum())
            rows.append({"lost_fraction": frac, "mode": name, "ms": float(np.median(times))})
    ms = {(r["lost_fraction"], r["mode"]): r["ms"] for r in rows}
    ratios = {f"{f:g}": {"sort/swap": ms[(f, "sort")] / ms[(f, "swap")],
                         "stable/swap": ms[(f, "stable")] / ms[(f, "swap")]}
              for f in (0.005, 0.05, 0.1, 0.5)}
    out = {"metric": "loss reordering time per call (ms), stable reordering at 5 % loss",
           "value": ms[(0.05, "stable")], "unit": "ms", "n_gpus": 1, "steps": reps, "warmup": 1,
           "ms_per_step": ms[(0.05, "stable")], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"loss reordering of {n:.0e} particles with losses at random "
                                  "slots (stable, the paper's sparse swap, sort by key)",
                      "particles": n},
           "table": rows, "ratios": ratios, "roofline": None}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported; the "
              "library tracks a beam on one device (a beam sharded by particle index over "
              "several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "surr":
        return surrogate_bench(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "compact":
        return compact_bench(args)
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = args.workload
    wake_mode = B.WAKE_FP32_MFMA if args.wake_mode == "fp32" else B.WAKE_FP64

    if wl in ("bc", "rfcw"):
        lat = inputs.bc_lattice() if wl == "bc" else inputs.rfcw_lattice()
        n = int(args.particles or 4_000_000)
        beam_kw = dict(n=n, seed=0, chirp=inputs.BC_CHIRP)
        p_ref, passes_per_step = inputs.BC_P0_EV, 1
        steps = args.steps or 50
        warm = args.warmup if args.warmup is not None else 5
        fresh = True
        cfg = {"workload": "linac bunch compressor: 4e6-particle chirped Gaussian beam, "
                           "8 x (RF cavity + 1024-bin wake step) + 2nd-order chicane"
                           if wl == "bc" else
                           "linac bunch compressor with transverse wakes: 4e6-particle chirped "
                           "Gaussian beam, 8 x (RF cavity + 1024-bin longitudinal and transverse "
                           "wake steps) + 2nd-order chicane",
               "particles": n, "elements_per_pass": len(lat),
               "wake_convolution": "fp32-mfma" if wake_mode == B.WAKE_FP32_MFMA else "fp64",
               "batch": "fresh device-resident beam per step"}
        sample = (n, 10)
    elif wl == "ring":
        lat = inputs.ring_lattice(seed=0)
        n = int(args.particles or 1_000_000)
        beam_kw = dict(n=n, seed=0)
        if args.sigma_scale != 1.0:
            beam_kw["sigmas"] = tuple(args.sigma_scale * v for v in inputs.BEAM_SIGMAS)
        p_ref, passes_per_step = 1e9, 1
        steps = args.steps or 20
        warm = args.warmup if args.warmup is not None else 2
        fresh = False
        cfg = {"workload": "storage ring: 1e6 particles, 40 cells of Yoshida-4 kick-drift "
                           "quads and sector bends, random thin sextupoles, Philox radiation "
                           "kick, elliptical aperture with compaction, moments every turn",
               "particles": n, "elements_per_pass": len(lat), "turns_per_step": 1}
        sample = (100_000, 40)
    else:  # fodo / roof
        lat = inputs.fodo_lattice(quad_order=args.quad_order)
        n = int(args.particles or (10_000 if wl == "fodo" else 10_000_000))
        beam_kw = dict(n=n, seed=0)
        if args.sigma_scale != 1.0:
            beam_kw["sigmas"] = tuple(args.sigma_scale * v for v in inputs.BEAM_SIGMAS)
        p_ref = 1e9
        passes_per_step = 10 if wl == "roof" else 100
        steps = args.steps or 5
        warm = args.warmup if args.warmup is not None else 1
        fresh = True
        cfg = {"workload": f"FODO channel: {n:.0e} particles, 10 cells (60 elements) per pass, "
                           f"{passes_per_step} passes per step"
                           + (", third-order quadrupole maps" if args.quad_order == 3 else ""),
               "particles": n, "elements_per_pass": len(lat), "fusion_max_elements": args.fusion,
               "quad_order": args.quad_order}
        sample = (10_000, 100) if wl == "fodo" else (1_000_000, 10)

    L = B.Lattice(lat)
    d = inputs.gaussian_beam(**beam_kw)
    template = B.Beam.from_inputs(d)
    ws = B.Workspace(n)
    # two timed regions of `steps` steps each: the first, without per-kernel
    # events (an event between two kernels stalls the queue for a few us), gives
    # the throughput; the second, with HIP events around every fused run on the
    # same stream, gives the run kernel's average duration for the roofline
    nb = (warm + 2 * steps) if fresh else 1
    beams = []
    for _ in range(nb):
        b = B.Beam.__new__(B.Beam)
        b.n = n
        b.z = template.z.clone()
        b.id = template.id.clone()
        b.lost_at = template.lost_at.clone()
        b.n_alive = template.n_alive.clone()
        beams.append(b)
    mom = torch.zeros((max(passes_per_step, 1), 28), dtype=torch.float64, device="cuda")
    use_mom = wl == "ring"
    stream = torch.cuda.current_stream()

    def one_step(i):
        b = beams[i if fresh else 0]
        fp = 0 if fresh else i * passes_per_step
        B.track(b, L, passes_per_step, ws, seed=7, first_pass=fp, p_ref=p_ref,
                moments=mom if use_mom else None, wake_mode=wake_mode,
                max_elems_per_launch=args.fusion, stream=stream)

    def timed(i0, i1):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for i in range(i0, i1):
            one_step(i)
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    for i in range(warm):
        one_step(i)
    torch.cuda.synchronize()
    ms_total = timed(warm, warm + steps)
    B.profile_enable(True)
    timed(warm + steps, warm + 2 * steps)
    run_ms, run_launches = B.profile_read(0)
    B.profile_enable(False)

    def steps_of(i0, i1):
        """exact particle-element steps of steps [i0, i1)"""
        if fresh:
            tot = 0.0
            for i in range(i0, i1):
                la = beams[i].lost_at.cpu().numpy()
                tot += element_steps(lat, passes_per_step, n, la, 0)
            return tot
        # a continuing beam: count survivors per turn from the loss records
        la = beams[0].lost_at.cpu().numpy()
        first = i0 * passes_per_step
        last = i1 * passes_per_step
        nel = len(lat)
        lp = la >> 32
        lost = la >= 0
        alive_then = float((la < 0).sum()) + float((lost & (lp >= last)).sum())
        tot = alive_then * (last - first) * nel
        inside = lost & (lp >= first) & (lp < last)
        pl = lp[inside] - first
        el = la[inside] & 0xFFFFFFFF
        return tot + float((pl * nel + el + 1).sum())

    total_steps = steps_of(warm, warm + steps)
    value = total_steps / (ms_total / 1e3)
    prof_steps = steps_of(warm + steps, warm + 2 * steps)

    # roofline of the dominant kernel (fused element run)
    plan = launches_of(lat, 16, args.fusion)
    bytes_per_pass = 0.0
    launches_per_pass = 0.0
    for j, (e0, e1, npass) in enumerate(plan):
        nxt = plan[(j + 1) % len(plan)][0] if len(plan) > 1 else None
        next_wake = nxt is not None and lat[nxt].kind in WAKES and (j + 1 < len(plan))
        per = run_mask_bytes(lat, e0, e1, moments=(use_mom and e1 == len(lat)),
                             next_wake=next_wake)
        if npass > 1:
            bytes_per_pass += per / npass
            launches_per_pass += 1.0 / npass
        else:
            bytes_per_pass += per
            launches_per_pass += 1.0
    alive_mean = prof_steps / (steps * passes_per_step * len(lat))
    alg_bytes_per_launch = alive_mean * bytes_per_pass / launches_per_pass
    avg_ms = run_ms / max(run_launches, 1)
    achieved = alg_bytes_per_launch / (avg_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "kernel": "trk::k_run (fused element run)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": TRAFFIC_PER_LAUNCH.get((wl, args.fusion)) if args.quad_order == 2 else None,
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": run_launches,
            "alg_bytes_per_launch": round(alg_bytes_per_launch)}
    # a launch whose FP64 work per byte exceeds the machine balance is bound by
    # the FP64 vector units: report it against their peak instead
    fkey = wl
    if wl in ("fodo", "roof"):
        fkey = "fodo3" if args.quad_order == 3 else "fodo"
    fpp = FP64_FLOP_PER_STEP.get(fkey)
    if fpp is not None:
        steps_per_launch = prof_steps / max(run_launches, 1)
        flops = fpp * steps_per_launch
        if flops / max(alg_bytes_per_launch, 1.0) > FP64_PEAK_TFLOPS / (HBM_PEAK_GBS / 1e3):
            ach = flops / (avg_ms / 1e3) / 1e12
            roof.update({"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                         "traffic": None, "alg_flops_per_launch": flops,
                         "fp64_flops_per_element_step": fpp})

    out = {"metric": "particle·element steps/s (FP64 tracking)", "value": value,
           "unit": "particle·element steps/s", "n_gpus": 1, "steps": steps,
           "warmup": warm, "ms_per_step": ms_total / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": cfg, "roofline": roof}
    if not args.no_cpu_baseline:
        sn, sp = sample
        cv, cdt, cores = cpu_baseline(lat, beam_kw, sp, p_ref, sn)
        out["cpu_baseline"] = {"value": cv, "unit": "particle·element steps/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"{sn} particles of the same workload, {sp} passes, "
                                         f"{cdt:.1f} s wall"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()

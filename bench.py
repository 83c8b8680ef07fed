#!/usr/bin/env python3
"""Throughput benchmark: particle-element steps per second on one MI355X.

Headline workload (the JSON line's `value`): the linac bunch compressor --
4e6 particles of a chirped 6D Gaussian beam through 8 zero-length RF
cavities, each followed by the longitudinal wake step (1024-bin histogram of
s, FP32 matrix-core causal convolution with a resonator wake, interpolated
energy kick), then a second-order chicane map (17 elements per pass).  One
step = one pass of a fresh, already device-resident batch.  A
particle-element step is one element applied to one particle alive at its
entry.

The default run adds, under "configs", every other configured workload with
its own roofline and CPU-oracle baseline: the FODO channel (1e4 particles,
100 passes), the FODO channel at 1e7 particles one element per launch (HBM
bound) and whole passes fused (FP64 bound), the storage ring as one
1000-turn call (1e6 particles, moments every turn), the batched scan (256
ring variants, 200 turns, against the variants tracked one at a time), the
bunch compressor at 4e7 particles (beyond the 256 MB Infinity Cache), the
sweep of the particle count from 1e4 to 1e7, the fused-against-separate
moment reductions and the learned section surrogate.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--headline-only]

Rooflines: the dominant kernel's duration comes from start and stop events
that its own dispatch packet records (hipExtLaunchKernel), accumulated over
a timed region on the kernel's stream; the algorithmic bytes or flops per
launch are stated per workload.  `--workload ceilings` measures the box's
copy, read and FP64 FMA ceilings; `--workload copycal` is a plain copy of
known size for calibrating the HBM byte counters.
"""
import argparse
import json
import os
import subprocess
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
TRAFFIC_PER_LAUNCH = {("bc", 0): 101936697, ("roof", 1): 734090445}
# FP64 vector peak (dense, FMA = 2 flops) and the FP64 flops of one
# particle-element step of each lattice: SQ_INSTS_VALU_FLOPS_FP64 (2 FMA + MUL
# + ADD + TRANS per wave instruction) x 64 lanes over the exact steps of a
# run in which nobody is lost (profiles/k_run_fp64_flops.md)
FP64_PEAK_TFLOPS = 78.6
FP64_FLOP_PER_STEP = {"ring": 135.8, "fodo": 60.0, "fodo3": 72.7}
BF16_PEAK_TFLOPS = 2500.0
STEP_UNIT = "particle·element steps/s"
KINDS = ("bc", "rfcw", "ring", "fodo", "roof", "surr", "batch", "compact", "sweep",
         "ablation", "ceilings", "copycal")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="bc", choices=KINDS)
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: skip the nested configurations")
    ap.add_argument("--epochs", type=int, default=200, help="surrogate training epochs")
    ap.add_argument("--precision", default="bf16x2", choices=["bf16", "bf16x2"])
    ap.add_argument("--margin", type=float, default=0.8, help="surrogate gate margin")
    ap.add_argument("--wake-mode", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--fusion", type=int, default=0, help="max elements per launch (roof)")
    ap.add_argument("--quad-order", type=int, default=2, choices=[2, 3],
                    help="fodo/roof: track the quadrupoles with second- or third-order maps")
    ap.add_argument("--turns", type=int, default=None, help="ring: turns per call; batch: turns")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--particles", type=float, default=None)
    ap.add_argument("--sigma-scale", type=float, default=1.0,
                    help="scale the Gaussian beam's sigmas (0.1: nobody is lost)")
    ap.add_argument("--mib", type=int, default=1024, help="copycal: MiB copied")
    ap.add_argument("--ppt", type=int, default=0,
                    help="particles per thread of the fused runs (0: automatic)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ counting
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


# ------------------------------------------------------------------ CPU oracle
def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lattice, beam_kw, passes, p_ref, n_all, n_one=None, seed=0, what=""):
    """The CPU oracle on the workload's own lattice and beam (the first
    n_all particles of it; particles are independent and their random kicks
    keyed by id), timed on all host threads and on one thread (the first
    n_one particles).  Returns the cpu_baseline object."""
    import oracle
    from paper_1710_07350_amd import inputs
    kw = {k: v for k, v in beam_kw.items() if k != "n"}
    threads = oracle.get_threads()

    def one(n):
        d = inputs.gaussian_beam(n, **kw)
        b = oracle.Beam.from_inputs(d, n0=beam_kw.get("n"))
        t0 = time.perf_counter()
        oracle.track(b, lattice, passes, p_ref=p_ref, seed=seed)
        dt = time.perf_counter() - t0
        return element_steps(lattice, passes, n, b.lost_at, 0) / dt, dt

    v_all, t_all = one(n_all)
    n_one = n_one or n_all
    oracle.set_threads(1)
    try:
        v_one, t_one = one(n_one)
    finally:
        oracle.set_threads(threads)
    return {"value": v_all, "unit": STEP_UNIT, "cores": threads, "kind": "oracle",
            "value_1core": v_one, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{what}: {n_all} particles on {threads} threads ({t_all:.1f} s), "
                      f"{n_one} on 1 thread ({t_one:.1f} s), {passes} passes each"}


# ------------------------------------------------------------------ tracking workloads
def track_workload(wl, args, n=None, steps=None, warm=None, fusion=None, passes=None,
                   cpu=True, roof=True):
    """Time `steps` tracking steps of workload wl (bc, rfcw, fodo, roof, ring)
    after `warm` untimed ones; returns the result object (without the
    contract's outer fields when nested)."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    fusion = args.fusion if fusion is None else fusion
    wake_mode = B.WAKE_FP32_MFMA if args.wake_mode == "fp32" else B.WAKE_FP64
    sig = None
    if args.sigma_scale != 1.0:
        sig = tuple(args.sigma_scale * v for v in inputs.BEAM_SIGMAS)
    use_mom = False
    if wl in ("bc", "rfcw"):
        lat = inputs.bc_lattice() if wl == "bc" else inputs.rfcw_lattice()
        n = int(n or args.particles or 4_000_000)
        beam_kw = dict(n=n, seed=0, chirp=inputs.BC_CHIRP)
        p_ref, pps = inputs.BC_P0_EV, 1
        steps = steps or args.steps or 50
        warm = warm if warm is not None else (args.warmup if args.warmup is not None else 5)
        cfg = {"workload": (f"linac bunch compressor: {n:.0e}-particle chirped Gaussian beam, "
                            "8 x (RF cavity + 1024-bin wake step) + 2nd-order chicane")
               if wl == "bc" else
               (f"linac bunch compressor with transverse wakes: {n:.0e}-particle chirped "
                "Gaussian beam, 8 x (RF cavity + 1024-bin longitudinal and transverse wake "
                "steps) + 2nd-order chicane"),
               "particles": n, "elements_per_pass": len(lat),
               "wake_convolution": "fp32-mfma" if wake_mode == B.WAKE_FP32_MFMA else "fp64",
               "batch": "fresh device-resident beam per step"}
        cpu_n = (n, n) if n <= 4_000_000 else (4_000_000, 1_000_000)
    elif wl == "ring":
        lat = inputs.ring_lattice(seed=0)
        n = int(n or args.particles or 1_000_000)
        beam_kw = dict(n=n, seed=0)
        if sig:
            beam_kw["sigmas"] = sig
        p_ref = 1e9
        pps = int(passes or args.turns or 1000)
        steps = steps or args.steps or 2
        warm = warm if warm is not None else (args.warmup if args.warmup is not None else 1)
        use_mom = True
        cfg = {"workload": f"storage ring: {n:.0e} particles, {pps} turns in one call, 40 cells of "
                           "Yoshida-4 kick-drift quads and sector bends, random thin sextupoles, "
                           "Philox radiation kick, elliptical aperture with compaction, moments "
                           "every turn",
               "particles": n, "elements_per_pass": len(lat), "turns_per_call": pps,
               "batch": "fresh device-resident beam per call"}
        cpu_n = (2000, 500)
    else:  # fodo / roof
        lat = inputs.fodo_lattice(quad_order=args.quad_order)
        n = int(n or args.particles or (10_000 if wl == "fodo" else 10_000_000))
        beam_kw = dict(n=n, seed=0)
        if sig:
            beam_kw["sigmas"] = sig
        p_ref = 1e9
        pps = int(passes or (10 if wl == "roof" else 100))
        steps = steps or args.steps or 5
        warm = warm if warm is not None else (args.warmup if args.warmup is not None else 1)
        cfg = {"workload": f"FODO channel: {n:.0e} particles, 10 cells (60 elements) per pass, "
                           f"{pps} passes per step"
                           + (f", at most {fusion} elements per launch" if fusion else
                              ", whole passes fused")
                           + (", third-order quadrupole maps" if args.quad_order == 3 else ""),
               "particles": n, "elements_per_pass": len(lat), "fusion_max_elements": fusion,
               "quad_order": args.quad_order, "batch": "fresh device-resident beam per step"}
        cpu_n = (n, n) if n <= 10_000 else (100_000, 20_000)

    L = B.Lattice(lat)
    d = inputs.gaussian_beam(**beam_kw)
    template = B.Beam.from_inputs(d)
    del d
    ws = B.Workspace(n)
    nb = warm + 2 * steps
    beams = []
    for _ in range(nb):
        b = B.Beam.__new__(B.Beam)
        b.n = n
        b.z = template.z.clone()
        b.id = template.id.clone()
        b.lost_at = template.lost_at.clone()
        b.n_alive = template.n_alive.clone()
        beams.append(b)
    del template
    mom = torch.zeros((max(pps, 1), 28), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def one_step(i):
        B.track(beams[i], L, pps, ws, seed=7, first_pass=0, p_ref=p_ref,
                moments=mom if use_mom else None, wake_mode=wake_mode,
                max_elems_per_launch=fusion, run_ppt=args.ppt, stream=stream)

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
    # two timed regions of `steps` steps each: the first gives the
    # throughput, the second the run kernel's launch durations (start and
    # stop events recorded by each run's own dispatch, class 0)
    ms_total = timed(warm, warm + steps)
    B.profile_enable(True, classes=0b1101)
    timed(warm + steps, warm + 2 * steps)
    run_ms, run_launches = B.profile_read(0)
    hist_ms, hist_n = B.profile_read(2)
    conv_ms, conv_n = B.profile_read(3)
    B.profile_enable(False)

    def steps_of(i0, i1):
        tot = 0.0
        for i in range(i0, i1):
            tot += element_steps(lat, pps, n, beams[i].lost_at.cpu().numpy(), 0)
        return tot

    total_steps = steps_of(warm, warm + steps)
    value = total_steps / (ms_total / 1e3)
    prof_steps = steps_of(warm + steps, warm + 2 * steps)
    alive_end = int(beams[warm].n_alive.item())
    out = {"metric": "particle·element steps/s (FP64 tracking)", "value": value,
           "unit": STEP_UNIT, "steps": steps, "warmup": warm, "ms_per_step": ms_total / steps,
           "dtype": "f64", "config": cfg, "alive_after_step": alive_end}
    kernels = {"run": {"launches": run_launches, "avg_us": 1e3 * run_ms / max(run_launches, 1)}}
    if hist_n:
        kernels["histogram"] = {"launches": hist_n, "avg_us": 1e3 * hist_ms / hist_n}
    if conv_n:
        kernels["convolution"] = {"launches": conv_n, "avg_us": 1e3 * conv_ms / conv_n}
    out["kernel_time"] = kernels

    if roof:
        plan = launches_of(lat, 16, fusion)
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
        alive_mean = prof_steps / (steps * pps * len(lat))
        alg_bytes_per_launch = alive_mean * bytes_per_pass / launches_per_pass
        avg_ms = run_ms / max(run_launches, 1)
        achieved = alg_bytes_per_launch / (avg_ms / 1e3) / 1e9
        rf = {"bound": "hbm", "kernel": "trk::k_run (fused element run)",
              "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(achieved / HBM_PEAK_GBS, 4),
              "traffic": (TRAFFIC_PER_LAUNCH.get((wl, fusion)) if args.quad_order == 2
                          and n == (4_000_000 if wl == "bc" else 10_000_000) else None),
              "avg_launch_us": round(avg_ms * 1e3, 2), "launches": run_launches,
              "alg_bytes_per_launch": round(alg_bytes_per_launch),
              "timing": "start/stop events recorded by each launch's dispatch packet"}
        fkey = wl
        if wl in ("fodo", "roof"):
            fkey = "fodo3" if args.quad_order == 3 else "fodo"
        fpp = FP64_FLOP_PER_STEP.get(fkey)
        if fpp is not None:
            steps_per_launch = prof_steps / max(run_launches, 1)
            flops = fpp * steps_per_launch
            # FP64 work per byte above the machine balance: bound by the
            # FP64 vector units
            if flops / max(alg_bytes_per_launch, 1.0) > FP64_PEAK_TFLOPS / (HBM_PEAK_GBS / 1e3):
                ach = flops / (avg_ms / 1e3) / 1e12
                rf.update({"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                           "traffic": None, "alg_flops_per_launch": flops,
                           "fp64_flops_per_element_step": fpp})
        out["roofline"] = rf
    del beams
    torch.cuda.empty_cache()
    if cpu and not args.no_cpu_baseline:
        log(f"{wl}: CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(lat, beam_kw, pps, p_ref, cpu_n[0], cpu_n[1],
                                           seed=7, what=f"{wl} workload")
    return out


# ------------------------------------------------------------------ surrogate
def surrogate_bench(args, n=None):
    """Train the section surrogate, then time plain tracking against
    gate + network + fallback on fresh particles of three distributions."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    n = int(n or args.particles or 10_000_000)
    prec = B.MLP_BF16X2 if args.precision == "bf16x2" else B.MLP_BF16
    margin, aper = args.margin, (10e-3, 5e-3)
    hw = 6.0 * np.array(inputs.BEAM_SIGMAS)
    sec = inputs.ring_lattice(seed=0)[:100]
    L = B.Lattice(sec)
    sur = B.Surrogate(L, hw, margin, aper)
    ws = sur.workspace(n)
    t0 = time.perf_counter()
    beam = B.Beam.empty(n)
    B.surrogate_sample(sur, 5, 0, beam, ws)
    u, r, npairs_t = B.surrogate_pairs(sur, beam, ws)
    npairs = int(npairs_t.item())
    D = B.surrogate_fit_scale(sur, r, npairs, ws)
    del beam
    t_pairs = time.perf_counter() - t0
    log(f"surrogate pairs: {npairs} in {t_pairs:.2f} s; D = {D}")
    inv = [1.0 / v if v > 0 else 0.0 for v in D]
    m = B.Mlp(inputs.mlp_init_params(21))
    batch = 8192
    mws = B.mlp_workspace(batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = B.mlp_train(m, u, r, inv, mws, batch=batch, epochs=args.epochs, lr0=2e-3,
                       lr_min=1e-5, seed=9, precision=prec, n_pairs=npairs).cpu().numpy()
    t_train = time.perf_counter() - t0
    log(f"surrogate training: {args.epochs} epochs in {t_train:.1f} s, loss {loss[0]:.3e} -> "
        f"{loss[-1]:.3e}")
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
        log(json.dumps(out))
        return out

    fresh = B.Beam.empty(n)
    B.surrogate_sample(sur, 63, 0, fresh, ws)
    fh = fresh.host()
    del fresh
    dom = one_set({"z": fh["z"], "id": fh["id"], "lost_at": fh["lost_at"]},
                  "fresh uniform points of the training domain (box and gate)")
    box = one_set(inputs.uniform_box_beam(n, seed=61, half_widths=hw), "uniform +-6 sigma box")
    gauss = one_set(inputs.gaussian_beam(n, seed=62), "Gaussian ring beam")
    flops = 2.0 * (6 * 256 + 2 * 256 * 256 + 256 * 6)
    ach = dom["admitted"] * flops / (dom["infer_ms"] / 1e3) / 1e12
    mx = dom["max_abs_error"]
    return {"metric": "surrogate speedup over plain tracking of the section",
            "value": dom["speedup"], "unit": "x", "steps": 5, "warmup": 1,
            "ms_per_step": dom["ms_surrogate"], "higher_is_better": True,
            "dtype": "bf16 network (" + args.precision + " activations), f64 linear part and "
                     "fallback",
            "config": {"workload": "learned surrogate of ring cells 0-9 (100 elements), "
                                   f"{n:.0e} fresh particles, gate margin {margin}",
                       "training_pairs": npairs, "epochs": args.epochs, "batch": batch,
                       "train_s": round(t_train, 2), "final_loss": float(loss[-1])},
            "error": {"max_m": max(mx["x"], mx["y"], mx["s"]), "max_rad": max(mx["xp"], mx["yp"]),
                      "meets_1e-6": max(mx.values()) <= 1e-6},
            "sets": [dom, box, gauss],
            "roofline": {"bound": "mfma", "kernel": "trk::k_surr_infer",
                         "achieved": round(ach, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / BF16_PEAK_TFLOPS, 4), "traffic": None}}


# ------------------------------------------------------------------ batches
def batch_bench(args, turns=None):
    """256 ring variants (own sextupoles, own seeds, log-uniform sizes in
    [1e3, 1e5]) in one persistent launch sequence (autotuned, hipGraph),
    against the same variants tracked one at a time with trk_track."""
    import torch
    from paper_1710_07350_amd import autotune
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs

    nvar = 256
    turns = int(turns or args.turns or 200)
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
    log(f"batch autotune: {tune} in {t_tune:.1f} s")
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
    tb = float(np.median([batched() for _ in range(2)]))
    res_b = work.host()
    # one at a time (timed once: the kernels are warm from a two-turn call)
    vb = [B.Beam.from_inputs(b) for b in beams]
    vws = [B.Workspace(int(n)) for n in sizes]
    vmom = [torch.zeros((turns, 28), dtype=torch.float64, device="cuda") for _ in range(nvar)]
    B.track(B.Beam.from_inputs(beams[0]), Ls[0], 2, vws[0], seed=int(seeds[0]), moments=vmom[0])
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record()
    for v in range(nvar):
        B.track(vb[v], Ls[v], turns, vws[v], seed=int(seeds[v]), moments=vmom[v])
    e.record()
    torch.cuda.synchronize()
    ts = a.elapsed_time(e)
    same = True
    for v in range(nvar):
        h = vb[v].host()
        sl = slice(seg[v], seg[v + 1])
        o1 = np.argsort(res_b["id"][sl], kind="stable")
        o2 = np.argsort(h["id"], kind="stable")
        same &= bool(np.array_equal(res_b["z"][:, sl][:, o1], h["z"][:, o2]) and
                     np.array_equal(res_b["lost_at"][sl][o1], h["lost_at"][o2]))
    steps = element_steps(lats[0], turns, int(seg[-1]), res_b["lost_at"], 0)
    out = {"metric": "particle·element steps/s (batched ring scan)",
           "value": steps / (tb / 1e3), "unit": STEP_UNIT, "steps": turns, "warmup": 1,
           "ms_per_step": tb / turns, "higher_is_better": True, "dtype": "f64",
           "config": {"workload": f"batched scan: {nvar} ring variants, {int(seg[-1])} particles "
                                  f"(log-uniform 1e3-1e5 per variant), {turns} turns, moments "
                                  "every turn, one graph-captured persistent launch sequence",
                      "tuning": tune, "autotune_s": round(t_tune, 2)},
           "sequential": {"value": steps / (ts / 1e3), "ms": ts},
           "batched_ms": tb, "speedup_vs_sequential": ts / tb,
           "variants_identical_to_sequential": same}
    fl = FP64_FLOP_PER_STEP["ring"] * steps
    ach = fl / (tb / 1e3) / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "trk::k_batch (persistent; whole batched call)",
                       "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": None,
                       "fp64_flops_per_element_step": FP64_FLOP_PER_STEP["ring"]}
    if not args.no_cpu_baseline:
        log("batch: CPU oracle ...")
        v0 = int(np.argmin(sizes))
        out["cpu_baseline"] = cpu_baseline(lats[v0], dict(n=int(sizes[v0]), seed=1000 + v0),
                                           turns, 1e9, int(sizes[v0]), min(int(sizes[v0]), 500),
                                           seed=int(seeds[v0]),
                                           what=f"batched scan, variant {v0}")
    return out


# ------------------------------------------------------------------ loss reorderings
def compact_bench(args):
    """The paper's comparison of loss reorderings (Sec. 2.5): time the stable
    reordering, the paper's sparse swap and the sort by key on 4e6 particles
    with 0.5, 5, 10 and 50 % of them lost at random slots."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs
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
    return {"metric": "loss reordering time per call (ms), stable reordering at 5 % loss",
            "value": ms[(0.05, "stable")], "unit": "ms", "steps": reps, "warmup": 1,
            "ms_per_step": ms[(0.05, "stable")], "higher_is_better": False, "dtype": "int64",
            "config": {"workload": f"loss reordering of {n:.0e} particles with losses at random "
                                   "slots (stable, the paper's sparse swap, sort by key)",
                       "particles": n},
            "table": rows, "ratios": ratios, "roofline": None}


# ------------------------------------------------------------------ sweeps and ablations
def sweep_bench(args):
    """Steps/s against the particle count (the paper's speed-up against N,
    Sec. 3): the bunch compressor pass and the FODO channel with whole passes
    fused, N = 1e4 ... 1e7."""
    rows = []
    for n in (10_000, 30_000, 100_000, 300_000, 1_000_000, 3_000_000, 10_000_000):
        for wl, passes in (("bc", 1), ("roof", 10)):
            r = track_workload(wl, args, n=n, steps=5, warm=2, passes=passes, fusion=0,
                               cpu=False, roof=False)
            rows.append({"workload": wl, "particles": n, "value": r["value"],
                         "ms_per_step": round(r["ms_per_step"], 4),
                         "run_kernel_us": round(r["kernel_time"]["run"]["avg_us"], 2)})
            log(json.dumps(rows[-1]))
    return {"metric": "particle·element steps/s against N", "unit": STEP_UNIT,
            "config": {"workload": "bunch compressor (one pass per step) and FODO channel (10 "
                                   "passes per step, whole passes fused), N from 1e4 to 1e7"},
            "table": rows}


def ablation_bench(args):
    """Moment reductions (Sec. 2.4): the ring at 1e6 particles, 32 turns, one
    turn per launch, with no moments, with the per-turn moments fused into
    the run kernel (shifted one-pass rows), with a separate two-pass
    moments call after every turn, and with the separate call on
    Kahan-compensated sums (the paper's optional compensated reductions).
    Also the cost of one standalone call of each on the 1e6-particle beam."""
    import torch
    from paper_1710_07350_amd import binding as B
    from paper_1710_07350_amd import inputs
    n, turns = int(args.particles or 1_000_000), 32
    lat = inputs.ring_lattice(seed=0)
    L = B.Lattice(lat)
    src = B.Beam.from_inputs(inputs.gaussian_beam(n, seed=0))
    ws = B.Workspace(n)
    mom = torch.zeros((turns, 28), dtype=torch.float64, device="cuda")

    def run(mode):
        b = src.clone()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        if mode in ("separate", "compensated"):
            f = B.moments if mode == "separate" else B.moments_compensated
            for t in range(turns):
                B.track(b, L, 1, ws, seed=7, first_pass=t)
                mom[t].copy_(f(b, ws))
        else:
            B.track(b, L, turns, ws, seed=7, passes_per_launch=1,
                    moments=mom if mode == "fused" else None)
        e.record()
        torch.cuda.synchronize()
        return a.elapsed_time(e)

    out = {}
    modes = ("none", "fused", "separate", "compensated")
    for mode in modes:  # warm-up (first launches, allocations)
        run(mode)
    for mode in modes * 3:
        out.setdefault(mode, []).append(run(mode))
    res = {m: float(np.median(v)) / turns for m, v in out.items()}

    def one_call(f):
        ts = []
        for _ in range(11):
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record()
            f(src, ws)
            e.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(e))
        return float(np.median(ts[1:]))
    return {"metric": "ms per ring turn (1e6 particles) by moment-reduction scheme", "unit": "ms",
            "config": {"workload": f"storage ring, {n:.0e} particles, {turns} turns, one turn "
                                   "per launch"},
            "ms_per_turn": res,
            "moment_cost_ms_per_turn": {k: res[k] - res["none"]
                                        for k in ("fused", "separate", "compensated")},
            "standalone_call_ms": {"plain": one_call(B.moments),
                                   "compensated": one_call(B.moments_compensated)}}


def ceilings_bench(args):
    """Measured copy, read and FP64 FMA ceilings of the box, beside the
    datasheet peaks: the library's probe kernels over 1 GiB arrays and FP64
    fma chains, median of 20 launches timed with HIP events."""
    import torch
    from paper_1710_07350_amd import binding as B

    def median_ms(fn, reps=20):
        st = torch.cuda.current_stream()
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(st)
            fn()
            b.record(st)
            b.synchronize()
            t.append(a.elapsed_time(b))
        return float(np.median(t))

    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for blocks in (4096, 16384, 65536, 131072):
        ms = median_ms(lambda: B.probe_stream(src, dst, 0, blocks))
        out[f"copy_TBps_{blocks}"] = round(2 * 8 * n / (ms * 1e-3) / 1e12, 3)
        ms = median_ms(lambda: B.probe_stream(src, dst, 2, blocks))
        out[f"copy_nt_TBps_{blocks}"] = round(2 * 8 * n / (ms * 1e-3) / 1e12, 3)
        ms = median_ms(lambda: B.probe_stream(src, dst, 1, blocks))
        out[f"read_TBps_{blocks}"] = round(8 * n / (ms * 1e-3) / 1e12, 3)
    iters = 4096
    for blocks in (2048, 8192):
        buf = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
        ms = median_ms(lambda: B.probe_fma(buf, iters, blocks))
        out[f"fp64_fma_TFLOPs_{blocks}"] = round(blocks * 256 * 8 * iters * 2 / (ms * 1e-3) / 1e12,
                                                 2)
    out["copy_TBps"] = max(v for k, v in out.items() if k.startswith("copy_"))
    out["read_TBps"] = max(v for k, v in out.items() if k.startswith("read_"))
    out["fp64_TFLOPs"] = max(v for k, v in out.items() if k.startswith("fp64_fma_"))
    return {"metric": "measured ceilings", "config": {"workload": "copy/read 1 GiB, FP64 fma"},
            "ceilings": out}


def copycal_bench(args):
    """A plain device-to-device copy of known size (three times), for
    calibrating the HBM byte counters rocprofv3 reports per dispatch."""
    import torch
    n = args.mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"metric": "copy calibration", "config": {"workload": f"copy {args.mib} MiB x 3"}}


# ------------------------------------------------------------------ main
def contract(out, n_gpus=1):
    """The fields every printed line carries."""
    base = {"metric": out.get("metric"), "value": out.get("value"), "unit": out.get("unit"),
            "n_gpus": n_gpus, "steps": out.get("steps"), "warmup": out.get("warmup"),
            "ms_per_step": out.get("ms_per_step"),
            "higher_is_better": out.get("higher_is_better", True), "scaling": "weak",
            "vs_baseline": None, "dtype": out.get("dtype"), "data": "synthetic"}
    for k, v in out.items():
        if k not in base:
            base[k] = v
    return base


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported; the "
              "library tracks a beam on one device (a beam sharded by particle index over "
              "several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = args.workload
    single = {"surr": surrogate_bench, "batch": batch_bench, "compact": compact_bench,
              "sweep": sweep_bench, "ablation": ablation_bench, "ceilings": ceilings_bench,
              "copycal": copycal_bench}
    if wl in single:
        print(json.dumps(contract(single[wl](args))))
        return
    if wl != "bc" or args.headline_only:
        print(json.dumps(contract(track_workload(wl, args))))
        return

    t_start = time.perf_counter()
    head = track_workload("bc", args)
    configs = {}

    def nested(name, fn):
        t0 = time.perf_counter()
        log(f"--- {name}")
        try:
            configs[name] = fn()
        except Exception as exc:       # one failing extra must not hide the headline
            configs[name] = {"error": f"{type(exc).__name__}: {exc}"}
        configs[name]["wall_s"] = round(time.perf_counter() - t0, 1)
        torch.cuda.empty_cache()

    sub = argparse.Namespace(**{**vars(args), "steps": None, "warmup": None, "particles": None,
                                "fusion": 0, "turns": None})
    nested("fodo_1e4", lambda: track_workload("fodo", sub, steps=5, warm=1))
    nested("roof_1e7_one_element_per_launch",
           lambda: track_workload("roof", sub, steps=3, warm=1, fusion=1))
    nested("roof_1e7_whole_pass", lambda: track_workload("roof", sub, steps=3, warm=1, fusion=0))
    nested("ring_1e6_1000_turns", lambda: track_workload("ring", sub))
    nested("batch_256_200_turns", lambda: batch_bench(sub))
    nested("bc_4e7", lambda: track_workload("bc", sub, n=40_000_000, steps=5, warm=1, cpu=False))
    nested("n_sweep", lambda: sweep_bench(sub))
    nested("moment_reductions", lambda: ablation_bench(sub))
    nested("surrogate", lambda: surrogate_bench(sub))
    head["configs"] = configs
    head["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(contract(head)))


if __name__ == "__main__":
    main()

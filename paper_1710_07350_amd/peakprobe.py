"""Measured ceilings of the GPU the library runs on, beside the datasheet
peaks the rooflines quote (HBM 8 TB/s, FP64 vector 78.6 TFLOP/s):

  python -m paper_1710_07350_amd.peakprobe

  copy   dst = src + 1 over 1 GiB arrays (2 GiB moved per launch), with
         cached and with non-temporal accesses
  read   per-workgroup sums of a 1 GiB array
  fma    binary64 fma chains, 8 per lane, on a grid filling every CU

Each figure is the median of 20 launches timed with HIP events on the
launching stream.
"""
import json


def _median_ms(fn, reps=20):
    import torch
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
    t.sort()
    return t[len(t) // 2]


def main():
    import torch
    from paper_1710_07350_amd import binding as B
    assert torch.cuda.is_available(), "peakprobe needs a GPU"
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for blocks in (4096, 16384, 65536, 131072):
        ms = _median_ms(lambda: B.probe_stream(src, dst, 0, blocks))
        out[f"copy_TBps_{blocks}"] = round(2 * 8 * n / (ms * 1e-3) / 1e12, 3)
        ms = _median_ms(lambda: B.probe_stream(src, dst, 2, blocks))
        out[f"copy_nt_TBps_{blocks}"] = round(2 * 8 * n / (ms * 1e-3) / 1e12, 3)
        ms = _median_ms(lambda: B.probe_stream(src, dst, 1, blocks))
        out[f"read_TBps_{blocks}"] = round(8 * n / (ms * 1e-3) / 1e12, 3)
    iters = 4096
    for blocks in (2048, 8192):
        buf = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
        ms = _median_ms(lambda: B.probe_fma(buf, iters, blocks))
        out[f"fp64_fma_TFLOPs_{blocks}"] = round(blocks * 256 * 8 * iters * 2 / (ms * 1e-3) / 1e12, 2)
    out["copy_TBps"] = max(v for k, v in out.items() if k.startswith("copy_"))
    out["read_TBps"] = max(v for k, v in out.items() if k.startswith("read_"))
    out["fp64_TFLOPs"] = max(v for k, v in out.items() if k.startswith("fp64_fma_"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()

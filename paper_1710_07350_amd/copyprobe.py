"""A plain device-to-device copy of known size, for calibrating the HBM byte
counters (FETCH_SIZE, WRITE_SIZE) that rocprofv3 reports per dispatch.

  python -m paper_1710_07350_amd.copyprobe [MiB]
"""
import sys


def main():
    import torch
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB three times")


if __name__ == "__main__":
    main()

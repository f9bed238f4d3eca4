"""Plain device copy of a known size, the calibration reference for HBM byte
counters (FETCH_SIZE / WRITE_SIZE read for a kernel that moves exactly
`--mib` MiB in and out).

    python paper_2508_18114_amd/copyprobe.py [--mib 256] [--reps 3]
"""
import argparse
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    import torch
    n = a.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        t0 = time.perf_counter()
        y.copy_(x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"copy {a.mib} MiB: {el * 1e3:.3f} ms, {2 * a.mib * (1 << 20) / el / 1e9:.1f} GB/s (read + write)",
              flush=True)


if __name__ == "__main__":
    main()

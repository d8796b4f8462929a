"""Plain device-to-device copy of known size, for scaling rocprofv3's
FETCH_SIZE / WRITE_SIZE counters to bytes (run it under `rocprofv3 --pmc`).

python -m paper_1804_02883_amd.calibrate_copy [MiB]
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x 5 (each copy reads {mib} MiB and writes {mib} MiB)", flush=True)


if __name__ == "__main__":
    main()

"""Reference copy for calibrating HBM byte counters (FETCH_SIZE / WRITE_SIZE).

Runs a plain device-to-device copy of a known size several times so that a
counter run over this program gives the counter's reading per byte actually
moved (``python -m paper_2211_10185_amd.calibrate``).
"""
import json
import sys

import torch


def main(mib: int = 1024, reps: int = 5):
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_call": n * 4, "copy_bytes_written_per_call": n * 4,
                      "calls": reps}), flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1024)

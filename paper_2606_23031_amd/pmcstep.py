"""Two fwd+bwd steps of the 1080p driving workload, then a 256 MiB device
copy used to calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE readings.

Run under ``rocprofv3 --pmc <counter> -- python -u pmcstep.py``."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import bench  # noqa: E402
from paper_2606_23031_amd import dv  # noqa: E402
from synth import make_config  # noqa: E402


def main():
    cfg = make_config(2, v_close=10.0)
    ctx = dv.dv_ctx_create(0)
    step = bench.Step(ctx, dv, cfg["scene"], cfg["views"], cfg["opts"])
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    x = torch.empty(64 << 20, device="cuda")
    y = torch.empty(64 << 20, device="cuda")
    x.fill_(1.0)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print("pmc step done", flush=True)


if __name__ == "__main__":
    main()

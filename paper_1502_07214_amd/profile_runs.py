"""Fixed workloads for rocprofv3 runs.

    python -m paper_1502_07214_amd.profile_runs copy    # plain device copy of 1 GiB, 3 times
    python -m paper_1502_07214_amd.profile_runs sweep   # the benchmark's sweep launches (L=12, 256 walkers)

`copy` calibrates the FETCH_SIZE / WRITE_SIZE counters: each copy moves exactly
2^30 bytes in and 2^30 bytes out of HBM, so counter / 2^30 is the factor that
turns the counters of other kernels into bytes.  `sweep` runs three
iterations of the benchmark job (10^4 sweeps of 256 walkers at L = 12, T = 2,
each followed by the histogram merge and weight update).
"""
from __future__ import annotations

import sys


def copy(nbytes: int = 1 << 30, reps: int = 3):
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x {reps}", flush=True)


def sweep(iterations: int = 3):
    import torch

    from . import MucaJob, workloads

    w = workloads.workload("l12_t2_w256")
    job = MucaJob(w["L"], w["T"], w["n_walkers"], seed=w["seed"], max_delta=1)
    for it in range(iterations):
        job.sweep(w["sweeps"])
        job.update_weights(job.reduce_hist())
        print(f"iteration {it} done", flush=True)
    torch.cuda.synchronize()
    job.free()


if __name__ == "__main__":
    {"copy": copy, "sweep": sweep}[sys.argv[1]]()

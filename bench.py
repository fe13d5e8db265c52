#!/usr/bin/env python3
"""Benchmark: BP3.5 collocated stiffness, N = 7, FP64, 32^3-element perturbed
hex mesh (E = 32768, 16.8M local DOFs, 6 geometric factors per node, lambda = 0).

One step = one application of the operator to a resident input vector
(y = S u, one launch of the BP3.5 kernel).  Prints ONE JSON line with GDOF/s,
the HBM roofline fraction of the kernel (algorithmic bytes / average kernel
time, timed with events on the stream the kernel runs on, against 8 TB/s), the
measured device-to-device copy roofline, and the FP64 CPU oracle timed on the
host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 7
GRID = 32


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def alg_bytes_bp35(N: int, E: int, sbytes: int = 8, ybytes: int = 8, nfactors: int = 6) -> int:
    """Algorithmic HBM bytes of one BP3.5 apply: u read once, each factor read
    once, y written once (lambda = 0, beta = 0)."""
    npn = (N + 1) ** 3
    return E * npn * (sbytes + ybytes + nfactors * sbytes)


def copy_roofline(fem, torch, nbytes: int, reps: int = 20) -> dict:
    """Device-to-device copy of nbytes/2 read + nbytes/2 written (the paper's
    empirical roofline): best of the streaming-copy kernel and hipMemcpyAsync."""
    half = (nbytes // 2) // 16 * 16
    src = torch.empty(half // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    out = {}
    for name in ("kernel", "memcpy"):
        for _ in range(3):
            if name == "kernel":
                fem.fem_stream_copy(src, dst, half)
            else:
                dst.copy_(src)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            if name == "kernel":
                fem.fem_stream_copy(src, dst, half)
            else:
                dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = 2 * half / (ms * 1e-3) / 1e9
    assert torch.equal(src, dst)
    del src, dst
    out["best"] = max(out["kernel"], out["memcpy"])
    return out


def measured_traffic(kernel_sources: list[str], record: str) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if the kernel's sources are unchanged since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for s in kernel_sources:
        with open(os.path.join(ROOT, "paper_1711_00903_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return float(rec["traffic_bytes_per_launch"])


def cpu_baseline(X, u, budget_s: float) -> dict:
    """The FP64 oracle (plain C, OpenMP over elements) on the host's cores,
    repeated over the first elements of the workload for about budget_s."""
    import oracle
    threads = oracle.set_threads(0)
    pb = oracle.Problem(N, X)
    G = pb.G_gll()
    E = X.shape[0]
    # size the sample so that one pass takes ~1/5 of the budget
    Es = min(E, 512)
    t0 = time.perf_counter()
    oracle.bp35(N, G[:Es], u[:Es])
    dt = time.perf_counter() - t0
    Es = int(min(E, max(512, Es * (budget_s / 5) / max(dt, 1e-6))))
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        oracle.bp35(N, G[:Es], u[:Es])
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end:
            break
    t = float(np.median(times))
    return {"value": Es * (N + 1) ** 3 / t / 1e9, "unit": "GDOF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {Es} of {E} elements of the same mesh and field, "
                      f"{len(times)} passes, median pass {t * 1e3:.1f} ms"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of CPU-oracle timing (0 disables the CPU leg)")
    ap.add_argument("--epb", type=int, default=0, help="elements per workgroup (0 = library default)")
    ap.add_argument("--grid-cap", type=int, default=0, help="workgroups at most (0 = uncapped)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the operator is element-local and shards by element ranges with no "
              f"communication).", file=sys.stderr)
        return 2

    import torch

    import workloads
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    fem.lib()
    torch.cuda.set_device(0)
    if args.epb or args.grid_cap:
        fem.fem_tune_set(fem.FEM_OP_BP35, N, fem.FEM_F64, args.epb, args.grid_cap)

    log(f"bench: BP3.5 N={N} E={GRID ** 3}: building inputs")
    X = workloads.element_vertices(GRID)
    E = X.shape[0]
    u = workloads.field(E, N + 1)
    dev = DeviceMesh(N, X, h=1.0 / GRID)
    ut = torch.from_numpy(u).cuda()
    y = torch.empty_like(ut)
    G, _ = dev.geometry(fem.FEM_QUAD_GLL, want_wJ=False)
    stream = torch.cuda.current_stream()

    def step():
        fem.fem_stiff_collocated_apply(N, E, dev.D1d, G, None, 0.0, ut, y, 0.0, fem.FEM_F64, 1.0,
                                       stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-launch kernel time: events on the kernel's own stream around each launch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        step()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
    ms_per_step = wall * 1e3 / args.steps
    log(f"bench: {args.steps} steps, {ms_per_step:.4f} ms/step wall, kernel {kern_ms:.4f} ms")

    epb = fem.fem_tune_get(fem.FEM_OP_BP35, N, fem.FEM_F64)[0]
    dofs = E * (N + 1) ** 3
    bytes_launch = alg_bytes_bp35(N, E)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    copy = copy_roofline(fem, torch, bytes_launch)
    log(f"bench: copy roofline {copy}")

    cpu = None
    if args.cpu_budget > 0:
        log("bench: timing the CPU oracle")
        cpu = cpu_baseline(X, u, args.cpu_budget)

    rec = {
        "metric": "BP3.5 N=7 GDOF/s (FP64, 32^3 perturbed hex mesh)",
        "value": dofs / (ms_per_step * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bp35_n7_e32768", "op": "BP3.5", "N": N, "E": E,
                   "dofs": dofs, "factors": 6, "lambda": 0.0, "storage": "f64",
                   "epb": epb,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(["bp35.hpp", "fem_device.hpp", "tiles.hpp", "launch.hpp"],
                                                 "bp35_n7_e32768_f64_traffic.json") if epb == 1 else None,
                     "kernel": f"bp35_kernel<{N + 1},{epb},double>", "kernel_ms": kern_ms,
                     "alg_bytes_per_launch": bytes_launch},
        "copy_roofline": {"GB/s": copy["best"], "kernel_GB/s": copy["kernel"],
                          "memcpy_GB/s": copy["memcpy"], "bytes": bytes_launch,
                          "frac_of_copy": achieved / copy["best"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

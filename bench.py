#!/usr/bin/env python3
"""Benchmark: BP3.5 collocated stiffness, N = 7, FP64, 32^3-element perturbed
hex mesh (E = 32768, 16.8M local DOFs, 6 geometric factors per node, lambda = 0).

One step = one application of the operator to a resident input vector
(y = S u, one launch of the BP3.5 kernel).  Prints ONE JSON line with GDOF/s,
the HBM roofline fraction of the kernel (algorithmic bytes / average kernel
time, timed with events on the stream the kernel runs on, against 8 TB/s), the
measured device-to-device copy roofline, and the FP64 CPU oracle timed on the
host's cores on a bounded sample of the same workload.

The record also carries two sub-records measured in the same run: ``small_case``
(BP1.0, N = 3, E = 512: cache-resident, time per apply) and ``cg`` (CG on
S + 4096 M at N = 7 on the 64^3 mesh to relative residual 1e-10: FP64 against
BF16-stored geometric data with FP64 vectors, and against iterative refinement
with an FP32 inner CG on BF16-stored geometric data; three solves each).

``--workload`` selects another single-operator workload with the same record
(BP1.0 or BP3.0, N = 7, on the 64^3 mesh); ``--cg``, ``--sweep`` and
``--batch`` run the solver, the roofline sweep and the ragged batch.
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

# single-operator workloads: (operator, N, grid edge); E = edge^3
BENCH_WORKLOADS = {
    "bp35_n7_e32768": ("BP35", 7, 32),
    "bp10_n7_e262144": ("BP10", 7, 64),
    "bp30_n7_e262144": ("BP30", 7, 64),
    # BP3.5 with the geometric factors formed in the kernel from the vertices
    "bp35v_n7_e32768": ("BP35V", 7, 32),
    # BP3.0 likewise (factors at the Gauss points from the vertices)
    "bp30v_n7_e262144": ("BP30V", 7, 64),
}
# the sources whose hash must match the committed HBM counters of a workload
KERNEL_SOURCES = {
    "BP35": ["bp35.hpp", "bp35t.hpp", "lines.hpp", "fem_device.hpp", "tiles.hpp", "launch.hpp"],
    "BP10": ["bp10.hpp", "bp10t.hpp", "bp10tp.hpp", "lines.hpp", "bp35.hpp", "bp35t.hpp", "fem_device.hpp", "tiles.hpp",
             "launch.hpp"],
    "BP30": ["bp30.hpp", "bp30t.hpp", "bp30t2.hpp", "lines.hpp", "bp35.hpp", "bp35t.hpp", "fem_device.hpp",
             "tiles.hpp", "launch.hpp"],
    "BP35V": ["bp35v.hip", "lines.hpp", "fem_device.hpp", "tiles.hpp", "launch.hpp"],
    "BP30V": ["bp30v.hip", "lines.hpp", "fem_device.hpp", "tiles.hpp", "launch.hpp"],
}
OP_LABEL = {"BP10": "BP1.0", "BP35": "BP3.5", "BP30": "BP3.0", "BP35V": "BP3.5 (factors from vertices)",
            "BP30V": "BP3.0 (factors from vertices)"}
FP64_PEAK_TFLOPS = 78.6
# FP64 flops per GLL point of the in-kernel factors (BP3.5 from vertices): a_r and
# a_s (12), three cross products (27), |J| (5), weights and 1/|J| (3), six dot
# products (30) and their scaling (6)
VERTEX_GEO_FLOPS = 83


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def copy_roofline(fem, torch, nbytes: int, reps: int = 20, settle_s: float = 0.0) -> dict:
    """Device-to-device copy of nbytes/2 read + nbytes/2 written (the paper's
    empirical roofline): best of the streaming-copy kernel and hipMemcpyAsync,
    each the mean over `reps` back-to-back copies between two events.  With
    settle_s > 0 the copy kernel first runs for about that long (untimed), so
    that what follows is measured at the clocks of a busy GPU."""
    half = (nbytes // 2) // 16 * 16
    src = torch.empty(half // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    out = {}
    if settle_s > 0:
        t_end = time.perf_counter() + settle_s
        while time.perf_counter() < t_end:
            for _ in range(10):
                fem.fem_stream_copy(src, dst, half)
            torch.cuda.synchronize()
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


LDS_MODES = ((0, "read_b64", 8), (1, "read_b128", 16), (2, "write_b64", 8), (3, "write_b128", 16))


def lds_roofline(fem, torch, workgroups: int = 1280, iters: int = 2000, reps: int = 5) -> dict:
    """Measured LDS bandwidth B_sh (the shared-memory term of the paper's
    empirical performance model, eq. sharedRoof): the library's LDS probe
    (fem_lds_bandwidth) with 1280 workgroups of 256 lanes (five per CU, all
    resident at once with 32 KiB of LDS each), timed with events over `reps`
    launches, per access width and direction."""
    sink = torch.empty(workgroups * 256, dtype=torch.float64, device="cuda")
    out = {"workgroups": workgroups, "iters": iters}
    for mode, name, width in LDS_MODES:
        for _ in range(2):
            fem.fem_lds_bandwidth(mode, workgroups, iters, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fem.fem_lds_bandwidth(mode, workgroups, iters, sink)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_GB/s"] = workgroups * 256 * iters * 16 * width / (ms * 1e-3) / 1e9
    assert torch.isfinite(sink).all()
    return out


def measured_traffic(kernel_sources: list[str], record: str, epb: int) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if the kernel's sources are unchanged since the counters were taken
    and the launch uses the same packing."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for s in kernel_sources:
        with open(os.path.join(ROOT, "paper_1711_00903_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("source_sha256") or rec.get("epb") != epb:
        return None
    return float(rec["traffic_bytes_per_launch"])


def cpu_baseline(op: str, Nb: int, X, u, budget_s: float) -> dict:
    """The FP64 oracle (plain C, OpenMP over elements) on the host's cores,
    repeated over the first elements of the workload for about budget_s."""
    import oracle
    threads = oracle.set_threads(0)
    E = X.shape[0]
    pb = oracle.Problem(Nb, X[:min(E, 16384)])
    apply = {"BP10": pb.mass, "BP35": pb.stiff35, "BP35V": pb.stiff35, "BP30": pb.stiff30, "BP30V": pb.stiff30}[op]
    apply(u[:min(E, 8)])   # geometry built outside the timing
    # size the sample so that one pass takes ~1/5 of the budget
    Es = min(E, 512)
    t0 = time.perf_counter()
    apply(u[:Es])
    dt = time.perf_counter() - t0
    Es = int(min(pb.E, max(512, Es * (budget_s / 5) / max(dt, 1e-6))))
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        apply(u[:Es])
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end:
            break
    t = float(np.median(times))
    return {"value": Es * (Nb + 1) ** 3 / t / 1e9, "unit": "GDOF/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {Es} of {E} elements of the same mesh and field, "
                      f"{len(times)} passes, median pass {t * 1e3:.1f} ms"}


# (name, mode, inner storage): FP64 CG; mixed precision with FP64 vectors and
# narrow geometric data; FP32 vectors and arithmetic with reliable updates
# (f32); and iterative refinement (mode 2: the FP32 inner CG restarted at
# every FP64 residual replacement) with FP32 vectors and u, G stored FP32,
# BF16 or FP16 (scaled)
CG_ARMS = [("fp64", 0, 0), ("f32g64", 1, 6), ("bf16g64", 1, 7), ("f16g64", 1, 8), ("f32", 1, 1),
           ("f32_ir", 2, 1), ("bf16g_ir", 2, 4), ("f16g_ir", 2, 5)]


def cg_rhs(dev, torch, workloads, E: int, Nq: int):
    """b = sin(pi x) sin(pi y) sin(pi z) + 1e-3 U[-1,1] at every local GLL node
    (noise seed 2017), built on the device from the library's node coordinates."""
    import math
    xyz = dev.node_coords()
    b = torch.sin(math.pi * xyz[..., 0]) * torch.sin(math.pi * xyz[..., 1]) * torch.sin(math.pi * xyz[..., 2])
    del xyz
    noise = torch.empty_like(b)
    for start, blk in workloads.field_chunked(E, Nq, seed=workloads.SEED_RHS_NOISE, chunk=1 << 15):
        noise[start:start + blk.shape[0]] = torch.from_numpy(blk).cuda()
    b = (b + 1e-3 * noise).contiguous()
    return b


def cg_arms(grid: int, lam: float, rtol: float, arm_names: list[str], solves: int = 1, max_iters: int = 20000,
            fusion: str = "auto", floor_iters: int = 0, history: bool = False, cg_delta: float = 0.1) -> dict:
    """Time to solution of (S + lambda M) x = b at N = 7 on the grid^3 mesh, per
    arm: FP64 CG, or mixed precision with the operator's geometric data stored
    narrow.  Every arm uses FP64 reliable updates and the same stopping rule on
    the FP64 true residual.  Each arm is solved `solves` times from x0 = 0; the
    record holds the median time, every solve's iterations, the library's final
    FP64 true residual, and speedups over the FP64 arm both in time to the
    tolerance and per iteration."""
    import torch

    import workloads
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh

    fem.lib()
    Ncg = 7
    X = workloads.element_vertices(grid)
    E = X.shape[0]
    log(f"cg: N={Ncg} E={E} lambda={lam}: building inputs")
    dev = DeviceMesh(Ncg, X, h=1.0 / grid)
    b = cg_rhs(dev, torch, workloads, E, Ncg + 1)
    arms = [a for a in CG_ARMS if a[0] in arm_names]
    for _, mode, prec in arms:   # all geometric data built before any timing
        dev.geometry(fem.FEM_QUAD_GLL, fem.FEM_F64, want_wJ=False)
        dev.geometry(fem.FEM_QUAD_GL, fem.FEM_F64, want_G=False, kind="wJ")
        if mode in (1, 2):
            dev.geometry(fem.FEM_QUAD_GLL, prec, want_wJ=False)
            dev.geometry(fem.FEM_QUAD_GL, prec, want_G=False, kind="wJ")
    torch.cuda.synchronize()
    out = {"workload": f"cg_n7_e{E}", "E": E, "N": Ncg, "dofs": E * (Ncg + 1) ** 3, "lambda": lam,
           "fusion": fusion, "solves_per_arm": solves, "arms": {}}
    tau = rtol
    if floor_iters > 0:
        # attainable FP64 accuracy: run FP64 CG far past convergence and take the
        # smallest true residual of its reliable updates
        x = torch.zeros_like(b)
        rep = dev.cg_solve(b, x, lam=lam, mode=0, rtol=1e-16, max_iters=floor_iters,
                           fusion=fem.FUSION_NAMES[fusion], history=4096)
        hist = rep.pop("history")
        floor = min(hist)
        out["floor"] = {"min_rel_res": floor, "updates": len(hist), "history": hist,
                        "iters": rep["iters"], "ms": rep["ms"]}
        log(f"cg: floor run {rep}; smallest true residual {floor:.3e}")
        tau = max(rtol, 2.0 * floor)
        del x
    out["tau"] = tau
    for name, mode, prec in arms:
        reps = []
        for k in range(solves):
            x = torch.zeros_like(b)
            maxit = max_iters if name != "f32" else min(max_iters, 4000)
            delta = cg_delta if mode == 2 else 0.1
            rep = dev.cg_solve(b, x, lam=lam, mode=mode, inner_prec=prec, rtol=tau, max_iters=maxit, delta=delta,
                               fusion=fem.FUSION_NAMES[fusion], history=4096 if history else 0)
            log(f"cg: {name} solve {k + 1}/{solves}: status {rep['status']} iters {rep['iters']} "
                f"rel_res {rep['rel_res']:.3e} {rep['ms']:.1f} ms")
            reps.append(rep)
            del x
        ms = [r["ms"] for r in reps]
        med = reps[int(np.argsort(ms)[len(ms) // 2])]
        rec = {"status": med["status"], "iters": [r["iters"] for r in reps], "ms": [r["ms"] for r in reps],
               "ms_median": float(np.median(ms)), "rel_res": [r["rel_res"] for r in reps],
               "reliable_updates": med["reliable_updates"], "hi_matvecs": med["hi_matvecs"],
               "ms_per_iter": float(np.median([r["ms"] / max(1, r["iters"]) for r in reps]))}
        if history:
            rec["history"] = med.get("history")
        out["arms"][name] = rec
        torch.cuda.empty_cache()
    fp = out["arms"].get("fp64")
    for name, rec in out["arms"].items():
        if fp and rec["status"] == 0 and fp["status"] == 0:
            rec["speedup_time_to_tau"] = fp["ms_median"] / rec["ms_median"]
            rec["speedup_per_iter"] = fp["ms_per_iter"] / rec["ms_per_iter"]
    del dev, b
    torch.cuda.empty_cache()
    return out


def run_cg(args) -> int:
    """Time to solution of (S + lambda M) x = b, N = 7, 64^3 elements (134M local
    DOFs), all arms (the oracle's re-evaluation of each final residual at this
    size is the GPU test tests/test_gpu_cg_full.py)."""
    out = cg_arms(args.cg_grid, args.cg_lambda, args.cg_rtol, args.cg_arms.split(","), solves=args.cg_solves,
                  max_iters=args.cg_max_iters, fusion=args.cg_fusion, floor_iters=args.cg_floor_iters,
                  history=args.cg_history, cg_delta=args.cg_ir_delta)
    print(json.dumps(out), flush=True)
    return 0


def run_pcg(args) -> int:
    """The assembled system Z^T (S + lambda M) Z x = b on the CG workload's mesh
    (N = 7, grid^3 elements; 90.5M global nodes at 64^3): Jacobi-PCG and
    unpreconditioned CG, FP64, to the same relative residual; b = sin(pi x)
    sin(pi y) sin(pi z) + 1e-3 U[-1,1] (seed 2017) at every global node.
    Reports iterations, time, time per iteration, and the assembled
    operator's own time per apply."""
    import torch

    import workloads
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh

    fem.lib()
    n, Np = args.cg_grid, 7
    X = workloads.element_vertices(n)
    E = X.shape[0]
    log(f"pcg: N={Np} E={E}: numbering and inverse map")
    gids, ng = workloads.global_numbering(n, Np)
    dev = DeviceMesh(Np, X, h=1.0 / n)
    dev.set_assembly(gids, ng)
    del gids
    xyz = dev.node_coords().reshape(-1, 3)
    first = dev._locals[dev._offsets[:-1].long()].long()      # first local copy of each global node
    xg = xyz[first]
    del xyz, first
    b = torch.sin(torch.pi * xg[:, 0]) * torch.sin(torch.pi * xg[:, 1]) * torch.sin(torch.pi * xg[:, 2])
    b = (b + 1e-3 * torch.from_numpy(workloads.global_noise(ng)).cuda()).contiguous()
    del xg
    out = {"workload": f"pcg_assembled_n7_e{E}", "E": E, "N": Np, "n_global": ng, "n_local": E * (Np + 1) ** 3,
           "cases": []}
    for lam in [float(v) for v in args.pcg_lambdas.split(",")]:
        # the assembled operator alone: time per apply
        u = torch.rand(ng, dtype=torch.float64, device="cuda")
        y = torch.empty_like(u)
        dev.assembled_apply(u, lam=lam, yg=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dev.assembled_apply(u, lam=lam, yg=y)
        e1.record()
        torch.cuda.synchronize()
        case = {"lambda": lam, "rtol": args.pcg_rtol, "apply_ms": e0.elapsed_time(e1) / 10, "arms": {}}
        del u, y
        for name, jacobi in (("jacobi_pcg", True), ("cg", False)):
            x = torch.zeros_like(b)
            rep = dev.pcg_solve(b, x, lam=lam, jacobi=jacobi, rtol=args.pcg_rtol, max_iters=args.cg_max_iters)
            rep["ms_per_iter"] = rep["ms"] / max(1, rep["iters"])
            log(f"pcg: lambda={lam} {name}: {rep}")
            case["arms"][name] = rep
            del x
        out["cases"].append(case)
    print(json.dumps(out), flush=True)
    return 0


def small_case(fem, torch, launches: int = 300) -> dict:
    """BP1.0, N = 3, 8^3 elements (E = 512, 1.04 MB per apply): cache-resident
    and launch-bound, so reported as time per apply, not as a fraction of HBM.
    Three views over `launches` applies each: back-to-back eager calls through
    the ABI (events around all of them), the same applies replayed from one
    captured graph, and per-launch event pairs (median kernel duration)."""
    import workloads
    from paper_1711_00903_amd.mesh import DeviceMesh

    Ns, n = 3, 8
    X = workloads.element_vertices(n)
    E = X.shape[0]
    dev = DeviceMesh(Ns, X, h=1.0 / n)
    ut = torch.from_numpy(workloads.field(E, Ns + 1)).cuda()
    y = torch.empty_like(ut)
    _, wJ = dev.geometry(fem.FEM_QUAD_GL, want_G=False, kind="wJ")
    stream = torch.cuda.Stream()

    def step():
        fem.fem_mass_apply(Ns, E, dev.I1d, wJ, ut, y, 0.0, fem.FEM_F64, 1.0, stream)

    with torch.cuda.stream(stream):
        for _ in range(50):
            step()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(launches):
            step()
        e1.record(stream)
        e1.synchronize()
        eager_us = e0.elapsed_time(e1) * 1e3 / launches
        descs = [dev.desc("BP10", ut, y) for _ in range(launches)]
        g = fem.BatchGraph(descs, lanes=1, stream=stream)
        for _ in range(3):
            g.launch(stream)
        stream.synchronize()
        e0.record(stream)
        g.launch(stream)
        e1.record(stream)
        e1.synchronize()
        graph_us = e0.elapsed_time(e1) * 1e3 / launches
        g.destroy()
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(launches)]
        for a, b in pairs:
            a.record(stream)
            step()
            b.record(stream)
        stream.synchronize()
        per = np.array([a.elapsed_time(b) * 1e3 for a, b in pairs])
    dofs = E * (Ns + 1) ** 3
    return {"workload": "bp10_n3_e512", "op": "BP1.0", "N": Ns, "E": E, "dofs": dofs, "dtype": "f64",
            "launches": launches, "us_per_apply_eager": eager_us, "us_per_apply_graph": graph_us,
            "kernel_us_median": float(np.median(per)), "kernel_us_min": float(per.min()),
            "GDOF/s_graph": dofs / (graph_us * 1e-6) / 1e9,
            "alg_bytes_per_apply": E * (2 * (Ns + 1) ** 3 + (Ns + 2) ** 3) * 8,
            "note": "cache-resident (1.04 MB per apply): launch-bound, no HBM roofline"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_sweep(args) -> int:
    """BP1.0 / BP3.5 / BP3.0 over N = 1..15 on the 64^3 mesh (E = 262144): every
    packing timed, the fastest kept (the tune table), throughput against the
    measured copy roofline."""
    import torch

    import workloads
    from paper_1711_00903_amd import fem, tune

    fem.lib()
    precs = [fem.PREC_NAMES[p] for p in args.sweep_precs.split(",")]
    Ns = [int(x) for x in args.sweep_ns.split(",")] if args.sweep_ns else list(range(1, 16))
    X = workloads.element_vertices(args.sweep_grid)
    copy = copy_roofline(fem, torch, 1 << 30, settle_s=0.5)
    log(f"sweep: copy roofline {copy}")
    lds = lds_roofline(fem, torch)
    log(f"sweep: LDS roofline {lds}")
    recs = tune.autotune(X, ops=tuple(args.sweep_ops.split(",")), Ns=Ns, precs=precs,
                         reps=args.sweep_reps, h=1.0 / args.sweep_grid, log=log)
    for r in recs:
        model_columns(r, copy["best"], lds)
    if args.tune_out:
        with open(args.tune_out, "w") as f:
            f.write(tune.table_text(recs))
    print(json.dumps({"workload": f"sweep_e{X.shape[0]}", "E": X.shape[0], "copy_roofline": copy,
                      "lds_roofline": lds, "records": recs}), flush=True)
    return 0


def model_columns(r: dict, copy_gbs: float, lds: dict) -> None:
    """The empirical model's two bounds on one apply (eqs. globalRoof and
    sharedRoof): HBM time = algorithmic bytes / B_copy; LDS time = the values
    the kernel's schedule reads and writes in LDS (s_r, s_w, tune.lds_values)
    over the measured 8-byte LDS read and write rates (the kernels' LDS
    accesses are 8 bytes wide or narrower).  The model time is the larger, so
    the rate bound is min(R_global, R_shared); the vector-ALU time of the
    algorithmic flops is reported beside them as a third ceiling."""
    from paper_1711_00903_amd import tune
    nb = tune.alg_bytes(r["op"], r["N"], r["E"], r["prec"])
    fam = tune.kernel_family(r["op"], r["N"], r["epb"], r["prec"])
    sr, sw = tune.lds_values(fam, r["N"])
    vb = 8 if r["prec"] in tune._F64_FIELDS else 4
    r["kernel"] = fam
    r["frac_of_copy"] = r["gbs"] / copy_gbs
    r["frac_of_peak"] = r["gbs"] / HBM_PEAK_GBS
    r["lds_bytes"] = r["E"] * (sr + sw) * vb
    r["t_hbm_ms"] = nb / (copy_gbs * 1e9) * 1e3
    r["t_lds_ms"] = r["E"] * (sr * vb / (lds["read_b64_GB/s"] * 1e9) + sw * vb / (lds["write_b64_GB/s"] * 1e9)) * 1e3
    # a third ceiling, not in the paper's model: the algorithmic flops (no
    # even-odd saving) at the vector peak of the arithmetic type
    r["t_alu_ms"] = tune.alg_flops(r["op"], r["N"], r["E"]) / ((FP64_PEAK_TFLOPS if vb == 8 else 157.3) * 1e12) * 1e3
    t = {"hbm": r["t_hbm_ms"], "lds": r["t_lds_ms"], "alu": r["t_alu_ms"]}
    r["bound"] = max(t, key=t.get)
    r["t_model_ms"] = t[r["bound"]]
    r["frac_of_model"] = r["t_model_ms"] / r["ms"]


def sweep_markdown(paths: list[str]) -> str:
    """Markdown summary of sweep records (bench.py --sweep JSON lines); a
    later file replaces the records of the (operator, N, precision) it
    covers.  The model columns are recomputed with each file's own copy and
    LDS rates."""
    from paper_1711_00903_amd import fem
    recs, notes = {}, []
    for path in paths:
        with open(path) as f:
            d = json.loads(f.read().strip().splitlines()[-1])
        notes.append(f"* `{os.path.basename(path)}`: copy {d['copy_roofline']['best']:.0f} GB/s, LDS 8-byte "
                     f"reads {d['lds_roofline']['read_b64_GB/s'] / 1e3:.1f} TB/s, writes "
                     f"{d['lds_roofline']['write_b64_GB/s'] / 1e3:.1f} TB/s")
        for r in d["records"]:
            model_columns(r, d["copy_roofline"]["best"], d["lds_roofline"])
            recs[(r["prec"], r["op"], r["N"])] = r
    names = {v: k for k, v in fem.PREC_NAMES.items()}
    out = ["Inputs (each with its measured rates):", *notes, ""]
    for prec in sorted({k[0] for k in recs}):
        out += [f"## {names[prec]}", "",
                "| N | op | kernel | epb / cap | ms | GB/s | % copy | % 8 TB/s | GDOF/s | t_HBM ms | t_LDS ms | "
                "t_ALU ms | bound | % of model |", "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
        for (p, op, N) in sorted(k for k in recs if k[0] == prec):
            r = recs[(p, op, N)]
            out.append(f"| {N} | {op} | {r['kernel']} | {r['epb']} / {r['grid_cap']} | {r['ms']:.4f} | "
                       f"{r['gbs']:.0f} | {100 * r['frac_of_copy']:.0f}% | {100 * r['frac_of_peak']:.0f}% | "
                       f"{r['gdofs']:.1f} | {r['t_hbm_ms']:.4f} | {r['t_lds_ms']:.4f} | {r['t_alu_ms']:.4f} | {r['bound']} | "
                       f"{100 * r['frac_of_model']:.0f}% |")
        out.append("")
    return "\n".join(out)


def run_case(args) -> int:
    """One operator at one degree and storage precision on the sweep mesh
    (64^3 by default): warm-up, then K back-to-back applies timed with events,
    for rocprofv3 kernel traces and counters of a single kernel."""
    import torch

    import workloads
    from paper_1711_00903_amd import fem, tune
    from paper_1711_00903_amd.mesh import DeviceMesh, FIELD_DTYPE, out_dtype

    fem.lib()
    op, Nc, pname = args.case.split(":")
    Nc = int(Nc)
    prec = fem.PREC_NAMES[pname]
    X = workloads.element_vertices(args.sweep_grid)
    dev = DeviceMesh(Nc, X, h=1.0 / args.sweep_grid)
    E = dev.E
    u = torch.from_numpy(workloads.field(E, Nc + 1)).cuda().to(FIELD_DTYPE[prec])
    y = torch.empty((E, dev.np), dtype=out_dtype(prec), device="cuda")
    call = {"BP10": lambda: dev.mass(u, y=y, prec=prec), "BP35": lambda: dev.stiff35(u, y=y, prec=prec),
            "BP30": lambda: dev.stiff30(u, y=y, prec=prec)}[op]
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nb = tune.alg_bytes(op, Nc, E, prec)
    opid = fem.OP_NAMES[op]
    epb, cap = fem.fem_tune_get(opid, Nc, prec)
    print(json.dumps({"case": args.case, "E": E, "epb": epb, "grid_cap": cap,
                      "kernel": tune.kernel_family(op, Nc, epb or 1, prec), "ms": ms, "alg_bytes": nb,
                      "GB/s": nb / (ms * 1e-3) / 1e9, "GDOF/s": E * dev.np / (ms * 1e-3) / 1e9}), flush=True)
    return 0


def run_batch(args) -> int:
    """Ragged batch: 64 independent meshes (N ~ U{1..15}, E log-uniform in
    [64, 32768], operator uniform over BP1.0 / BP3.5 / BP3.0; seed 355), FP64
    and FP32 storage.  Times one eager enqueue of all applies on one stream
    (fem_batch_apply) against one replay of the captured graph
    (fem_batch_graph_*) with 1, 4 and 8 lanes, each with the tuned packing of
    its (operator, N, precision)."""
    import torch

    import workloads
    from paper_1711_00903_amd import fem, tune
    from paper_1711_00903_amd.mesh import DeviceMesh, FIELD_DTYPE, out_dtype

    fem.lib()
    spec = workloads.ragged_batch(args.batch_count)
    stream = torch.cuda.Stream()   # graph capture needs a stream other than the legacy default one
    devs = []
    for m in spec:
        X = workloads.element_vertices(m.n, E=m.E, seed=m.mesh_seed)
        devs.append(DeviceMesh(m.N, X, h=1.0 / m.n))
    out = {"workload": f"ragged_batch_{len(spec)}",
           "meshes": [dict(op=m.op, N=m.N, E=m.E) for m in spec], "precs": {}}

    def timed(fn, reps):
        for _ in range(2):
            fn()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        t1.synchronize()
        return t0.elapsed_time(t1) / reps

    for pname in args.batch_precs.split(","):
        prec = fem.PREC_NAMES[pname]
        descs, keep = [], []
        nbytes = dofs = 0
        for m, dev in zip(spec, devs):
            u = torch.from_numpy(workloads.field(m.E, m.N + 1, seed=m.field_seed)).cuda().to(FIELD_DTYPE[prec])
            y = torch.zeros(u.shape, dtype=out_dtype(prec), device="cuda")
            keep += [u, y]
            descs.append(dev.desc(m.op, u, y, prec=prec))
            nbytes += tune.alg_bytes(m.op, m.N, m.E, prec)
            dofs += m.E * (m.N + 1) ** 3
        torch.cuda.synchronize()
        rec = {"alg_bytes": nbytes, "dofs": dofs}
        rec["eager_ms"] = timed(lambda: fem.fem_batch_apply(descs, stream), args.batch_reps)
        for lanes in (1, 4, 8):
            g = fem.BatchGraph(descs, lanes=lanes, stream=stream)
            rec[f"graph{lanes}_ms"] = timed(lambda: g.launch(stream), args.batch_reps)
            g.destroy()
        best = min(rec[k] for k in rec if k.endswith("_ms"))
        rec["best_GB/s"] = nbytes / (best * 1e-3) / 1e9
        rec["best_GDOF/s"] = dofs / (best * 1e-3) / 1e9
        rec["graph_speedup"] = rec["eager_ms"] / min(rec["graph1_ms"], rec["graph4_ms"], rec["graph8_ms"])
        log(f"batch {pname}: {rec}")
        out["precs"][pname] = rec
        del descs, keep
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="bp35_n7_e32768", choices=sorted(BENCH_WORKLOADS))
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of CPU-oracle timing on all host cores (0 disables the CPU leg)")
    ap.add_argument("--cpu-budget-1core", type=float, default=4.0,
                    help="seconds of CPU-oracle timing on one core (0 disables)")
    ap.add_argument("--epb", type=int, default=0, help="elements per workgroup (0 = library default)")
    ap.add_argument("--grid-cap", type=int, default=0, help="workgroups at most (0 = uncapped)")
    ap.add_argument("--no-cg", action="store_true", help="leave the CG sub-record out of the default record")
    ap.add_argument("--no-small-case", action="store_true", help="leave the small-case sub-record out")
    ap.add_argument("--cg", action="store_true", help="time the CG workload instead")
    ap.add_argument("--cg-grid", type=int, default=64)
    ap.add_argument("--cg-rtol", type=float, default=1e-10)
    ap.add_argument("--cg-lambda", type=float, default=1.0,
                    help="mass coefficient of A = S + lambda M (1/h^2 = 4096 makes 1e-10 attainable in FP64)")
    ap.add_argument("--cg-floor-iters", type=int, default=0,
                    help="first run FP64 CG this long and set the tolerance to max(rtol, 2 x floor)")
    ap.add_argument("--cg-max-iters", type=int, default=20000)
    ap.add_argument("--cg-arms", default="fp64,f32g64,bf16g64,f16g64,f32,f32_ir,bf16g_ir,f16g_ir")
    ap.add_argument("--cg-ir-delta", type=float, default=0.1,
                    help="residual reduction of each inner solve of the iterative-refinement arms")
    ap.add_argument("--cg-solves", type=int, default=1, help="solves per arm (the median is reported)")
    ap.add_argument("--cg-history", action="store_true", help="record each arm's true-residual history")
    ap.add_argument("--cg-fusion", default="auto", choices=["auto", "none", "onepass"],
                    help="kernel split of the CG iteration (fem_cg_fusion)")
    ap.add_argument("--pcg", action="store_true", help="Jacobi-PCG on the assembled operator (CG mesh)")
    ap.add_argument("--pcg-lambdas", default="1,4096")
    ap.add_argument("--pcg-rtol", type=float, default=1e-8)
    ap.add_argument("--lds", action="store_true", help="measure the LDS bandwidth (B_sh) and exit")
    ap.add_argument("--sweep", action="store_true", help="roofline sweep over N and autotune")
    ap.add_argument("--sweep-grid", type=int, default=64)
    ap.add_argument("--sweep-precs", default="f64")
    ap.add_argument("--sweep-ns", default="")
    ap.add_argument("--sweep-ops", default="BP10,BP35,BP30")
    ap.add_argument("--sweep-reps", type=int, default=10)
    ap.add_argument("--tune-out", default="")
    ap.add_argument("--sweep-md", default="",
                    help="comma-separated sweep JSON files: print their merged markdown summary and exit")
    ap.add_argument("--case", default="",
                    help="OP:N:PREC (e.g. BP30:10:f64): K applies of that operator's tuned kernel on the "
                         "--sweep-grid mesh, for profiling; prints the mean kernel time")
    ap.add_argument("--batch", action="store_true", help="ragged batch: eager vs captured graph")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-precs", default="f64,f32")
    ap.add_argument("--batch-reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the operator is element-local and shards by element ranges with no "
              f"communication).", file=sys.stderr)
        return 2
    if args.lds:
        import torch
        from paper_1711_00903_amd import fem
        fem.lib()
        copy = copy_roofline(fem, torch, 1 << 30, settle_s=0.5)
        print(json.dumps({"lds_roofline": lds_roofline(fem, torch), "copy_roofline": copy}), flush=True)
        return 0
    if args.sweep_md:
        print(sweep_markdown(args.sweep_md.split(",")))
        return 0
    if args.sweep:
        return run_sweep(args)
    if args.batch:
        return run_batch(args)
    if args.cg:
        return run_cg(args)
    if args.pcg:
        return run_pcg(args)
    if args.case:
        return run_case(args)

    import torch

    import workloads
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    fem.lib()
    torch.cuda.set_device(0)
    workload = args.workload
    op, Nb, grid = BENCH_WORKLOADS[workload]
    opid = fem.OP_NAMES[op] if op in fem.OP_NAMES else None
    if opid is not None and (args.epb or args.grid_cap):
        fem.fem_tune_set(opid, Nb, fem.FEM_F64, args.epb, args.grid_cap)

    log(f"bench: {OP_LABEL[op]} N={Nb} E={grid ** 3}: building inputs (library {fem.fem_build_id()})")
    X = workloads.element_vertices(grid)
    E = X.shape[0]
    u = workloads.field(E, Nb + 1)
    dev = DeviceMesh(Nb, X, h=1.0 / grid)
    ut = torch.from_numpy(u).cuda()
    y = torch.empty_like(ut)
    stream = torch.cuda.current_stream()
    if op == "BP35":
        G, _ = dev.geometry(fem.FEM_QUAD_GLL, want_wJ=False)

        def step():
            fem.fem_stiff_collocated_apply(Nb, E, dev.D1d, G, None, 0.0, ut, y, 0.0, fem.FEM_F64, 1.0, stream)
    elif op == "BP35V":
        def step():
            fem.fem_stiff_collocated_vertex_apply(Nb, E, dev.D1d, dev.X, 0.0, ut, y, 0.0, stream)
    elif op == "BP30V":
        def step():
            fem.fem_stiff_dealiased_vertex_apply(Nb, E, dev.I1d, dev.Dgl, dev.X, 0.0, ut, y, 0.0, stream)
    elif op == "BP10":
        _, wJ = dev.geometry(fem.FEM_QUAD_GL, want_G=False, kind="wJ")

        def step():
            fem.fem_mass_apply(Nb, E, dev.I1d, wJ, ut, y, 0.0, fem.FEM_F64, 1.0, stream)
    else:
        G, _ = dev.geometry(fem.FEM_QUAD_GL, want_wJ=False)

        def step():
            fem.fem_stiff_dealiased_apply(Nb, E, dev.I1d, dev.Dgl, G, None, 0.0, ut, y, 0.0, fem.FEM_F64,
                                          1.0, stream)

    from paper_1711_00903_amd import tune
    dofs = E * (Nb + 1) ** 3
    # algorithmic bytes: u and y once, plus the stored factors (or the 8 vertices)
    bytes_launch = (16 * dofs + 192 * E) if op in ("BP35V", "BP30V") else tune.alg_bytes(op, Nb, E, fem.FEM_F64)
    # copy roofline before the timed region; its first half second (untimed)
    # brings the GPU to the clocks it runs at under load
    copy_before = copy_roofline(fem, torch, bytes_launch, settle_s=0.5)
    log(f"bench: copy roofline before {copy_before}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed region: K back-to-back launches, bracketed by HIP events on the
    # kernel's own stream (average launch duration) and by the host clock
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    log(f"bench: {args.steps} steps, {ms_per_step:.4f} ms/step wall, kernel {kern_ms:.4f} ms (events over the loop)")

    # per-launch distribution, after the timed region: an event pair around each
    # launch (serialises the dispatches, so each includes the dispatch gap)
    npl = max(args.steps, 50)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(npl)]
    for s, e in pairs:
        s.record(stream)
        step()
        e.record(stream)
    torch.cuda.synchronize()
    per = np.array([s.elapsed_time(e) for s, e in pairs])
    # the same K launches replayed from one captured graph (no host in the
    # loop): separates the kernels' own time from what the eager dispatch of
    # dependent launches adds between them
    graph_ms = None
    if op in ("BP35", "BP10", "BP30"):
        gstream = torch.cuda.Stream()
        descs = [dev.desc(op, ut, y) for _ in range(args.steps)]
        g = fem.BatchGraph(descs, lanes=1, stream=gstream)
        for _ in range(2):
            g.launch(gstream)
        gstream.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(gstream)
        g.launch(gstream)
        g1.record(gstream)
        g1.synchronize()
        graph_ms = g0.elapsed_time(g1) / args.steps
        g.destroy()
        log(f"bench: {args.steps} launches from one graph: {graph_ms:.4f} ms per launch")
    copy_after = copy_roofline(fem, torch, bytes_launch)
    log(f"bench: copy roofline after {copy_after}")
    copy_best = max(copy_before["best"], copy_after["best"])

    if opid is None:
        epb = 1
    else:
        epb = fem.fem_tune_get(opid, Nb, fem.FEM_F64)[0] or fem.fem_supported_epb(opid, Nb, fem.FEM_F64)[0]
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    del ut, y
    torch.cuda.empty_cache()

    small = None
    if not args.no_small_case:
        log("bench: small case (BP1.0 N=3 E=512)")
        small = small_case(fem, torch)
        log(f"bench: small case {small}")

    cg = None
    if not args.no_cg:
        dev.drop_geometry()
        del dev
        torch.cuda.empty_cache()
        cg = cg_arms(64, 4096.0, 1e-10, ["fp64", "bf16g64", "bf16g_ir"], solves=3)
        log(f"bench: cg {json.dumps(cg)}")

    cpu = None
    if args.cpu_budget > 0:
        log("bench: timing the CPU oracle")
        cpu = cpu_baseline(op, Nb, X, u, args.cpu_budget)
        cpu["cpu_model"] = cpu_model()
        if args.cpu_budget_1core > 0:
            import oracle
            threads = oracle.set_threads(0)
            oracle.set_threads(1)
            one = cpu_baseline(op, Nb, X, u, args.cpu_budget_1core)
            oracle.set_threads(threads)
            cpu["value_1core"] = one["value"]
            cpu["sample_1core"] = one["sample"]

    kname = {"BP35": f"bp35_kernel<{Nb + 1},{epb},double,double>",
             "BP35V": f"bp35v_kernel<{Nb + 1}>",
             "BP30V": f"bp30v_kernel<{Nb + 1},double,double>",
             "BP10": f"bp10t_kernel<{Nb + 1},double,double>" if epb == 1
             else f"bp10_kernel<{Nb + 1},{epb},double,double>",
             "BP30": f"bp30t_kernel<{Nb + 1},double,double>" if epb == 1
             else f"bp30_kernel<{Nb + 1},{epb},double,double>"}[op]
    rec = {
        "metric": f"{OP_LABEL[op]} N={Nb} GDOF/s (FP64, {grid}^3 perturbed hex mesh)",
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
        "config": {"workload": workload, "op": OP_LABEL[op], "N": Nb, "E": E,
                   "dofs": dofs, "factors": 0 if op == "BP10" else 6, "lambda": 0.0, "storage": "f64",
                   "epb": epb,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(KERNEL_SOURCES[op], f"{workload}_f64_traffic.json", epb),
                     "kernel": kname, "kernel_ms": kern_ms,
                     "kernel_ms_source": "HIP events around the K timed launches on the kernel's stream",
                     "per_launch_ms": {"launches": npl, "median": float(np.median(per)), "mean": float(per.mean()),
                                       "min": float(per.min()), "max": float(per.max()),
                                       "source": "event pair around each launch, after the timed region"},
                     "graph_ms_per_launch": graph_ms,
                     "alg_bytes_per_launch": bytes_launch},
        "copy_roofline": {"GB/s": copy_best, "before_GB/s": copy_before["best"], "after_GB/s": copy_after["best"],
                          "kernel_GB/s": max(copy_before["kernel"], copy_after["kernel"]),
                          "memcpy_GB/s": max(copy_before["memcpy"], copy_after["memcpy"]), "bytes": bytes_launch,
                          "frac_of_copy": achieved / copy_best,
                          "frac_of_copy_uses": "the better of the copies measured before and after the timed region"},
        "cpu_baseline": cpu,
        "small_case": small,
        "cg": cg,
        "build_id": fem.fem_build_id(),
    }
    if op in ("BP35V", "BP30V"):
        # the factors are computed, not read: FP64 arithmetic is the bound to price against
        npts = (Nb + 1) ** 3 if op == "BP35V" else (Nb + 2) ** 3
        flops = E * (tune.alg_flops(op[:4], Nb, 1) + VERTEX_GEO_FLOPS * npts)
        tf = flops / (kern_ms * 1e-3) / 1e12
        rec["config"]["factors"] = "from vertices"
        rec["roofline"].update({"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": tf / FP64_PEAK_TFLOPS, "traffic": None, "alg_flops_per_launch": flops,
                                "fields_GB/s": achieved})
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

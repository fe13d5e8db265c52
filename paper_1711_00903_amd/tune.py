"""Autotuner of the element kernels' launch shape.

For each (operator, degree, precision) it times every supported number of
elements per workgroup on a device-resident mesh, keeps the fastest, and
writes the result as a tune table that ``fem_tune_load`` reads ("op N prec epb
grid_cap" per line).  The measured throughputs double as the roofline sweep
over N (GB/s of algorithmic traffic per apply).
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import fem
from .mesh import DeviceMesh, FIELD_DTYPE, out_dtype

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.txt")

_GEO_BYTES = {fem.FEM_F64: 8, fem.FEM_F32: 4, fem.FEM_BF16: 2, fem.FEM_F16: 2, fem.FEM_BF16G: 2,
              fem.FEM_F16G: 2, fem.FEM_F32G64: 4, fem.FEM_BF16G64: 2, fem.FEM_F16G64: 2}


def alg_bytes(op: str, N: int, E: int, prec: int) -> int:
    """Algorithmic HBM bytes of one apply (lambda = 0, beta = 0): fields read
    and written once, each geometric value read once."""
    nq, ng = N + 1, N + 2
    fb = torch.tensor([], dtype=FIELD_DTYPE[prec]).element_size()
    ob = torch.tensor([], dtype=out_dtype(prec)).element_size()
    gb = _GEO_BYTES[prec]
    geo = {"BP10": ng ** 3, "BP35": 6 * nq ** 3, "BP30": 6 * ng ** 3}[op] * gb
    return E * (nq ** 3 * (fb + ob) + geo)


def alg_flops(op: str, N: int, E: int) -> int:
    q, g = N + 1, N + 2
    f = {"BP10": 4 * (q ** 3 * g + q ** 2 * g ** 2 + q * g ** 3) + g ** 3,
         "BP35": 12 * q ** 4 + 17 * q ** 3,
         "BP30": 4 * (q ** 3 * g + q ** 2 * g ** 2 + q * g ** 3) + 12 * g ** 4 + 17 * g ** 3}[op]
    return E * f


def _time(fn, reps: int, stream) -> float:
    for _ in range(2):
        fn()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


def autotune(X: np.ndarray, ops=("BP10", "BP35", "BP30"), Ns=range(1, 16), precs=(fem.FEM_F64,),
             reps: int = 10, h: float | None = None, log=None, seed: int = 0) -> list[dict]:
    """Time every supported packing of each (op, N, prec) on the mesh X; returns
    one record per configuration with the fastest packing first-class."""
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    out = []
    for N in Ns:
        dev = DeviceMesh(N, X, h=h)
        E = dev.E
        for prec in precs:
            u = torch.empty((E, dev.np), dtype=torch.float32, device="cuda")
            gen.manual_seed(seed + N)
            u.uniform_(-1.0, 1.0, generator=gen)
            u = u.to(FIELD_DTYPE[prec])
            y = torch.empty((E, dev.np), dtype=out_dtype(prec), device="cuda")
            for op in ops:
                opid = fem.OP_NAMES[op]
                call = {"BP10": lambda: dev.mass(u, y=y, prec=prec, stream=stream),
                        "BP35": lambda: dev.stiff35(u, y=y, prec=prec, stream=stream),
                        "BP30": lambda: dev.stiff30(u, y=y, prec=prec, stream=stream)}[op]
                timings = {}
                try:
                    for epb in fem.fem_supported_epb(opid, N, prec):
                        fem.fem_tune_set(opid, N, prec, epb, 0)
                        timings[epb] = _time(call, reps, stream)
                finally:
                    fem.fem_tune_set(opid, N, prec, 0, 0)
                best = min(timings, key=timings.get)
                ms = timings[best]
                nbytes = alg_bytes(op, N, E, prec)
                rec = dict(op=op, N=N, prec=prec, E=E, epb=best, grid_cap=0, ms=ms,
                           gbs=nbytes / (ms * 1e-3) / 1e9, gdofs=E * dev.np / (ms * 1e-3) / 1e9,
                           tflops=alg_flops(op, N, E) / (ms * 1e-3) / 1e12,
                           all_ms={int(k): v for k, v in timings.items()})
                out.append(rec)
                if log:
                    log(f"tune {op} N={N} prec={prec}: epb {best} {ms:.4f} ms {rec['gbs']:.0f} GB/s "
                        f"{rec['gdofs']:.1f} GDOF/s  all {rec['all_ms']}")
            del u, y
        dev.drop_geometry()
        del dev
        torch.cuda.empty_cache()
    return out


def table_text(records: list[dict]) -> str:
    lines = ["# op N prec epb grid_cap   (measured on MI355X; fem_tune_load format)"]
    for r in records:
        lines.append(f"{fem.OP_NAMES[r['op']]} {r['N']} {r['prec']} {r['epb']} {r['grid_cap']}"
                     f"   # {r['op']} {r['ms']:.4f} ms {r['gbs']:.0f} GB/s")
    return "\n".join(lines) + "\n"


def load(path: str = TABLE) -> bool:
    """Apply a tune table file (the packaged MI355X table by default)."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        fem.fem_tune_load(f.read())
    return True

"""Autotuner of the element kernels' launch shape.

For each (operator, degree, precision) it times every supported number of
elements per workgroup -- and, for the column kernels, which loop over element
groups, every persistent grid size of GRID_CAPS -- on a device-resident mesh,
keeps the fastest, and writes the result as a tune table that ``fem_tune_load``
reads ("op N prec epb grid_cap" per line).  The line-per-lane kernels have one
launch shape each; their LDS layout and table placement per (operator, degree,
arithmetic) were chosen by measurement and are fixed in the kernels.  The measured throughputs double as the roofline sweep
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


_F64_FIELDS = (fem.FEM_F64, fem.FEM_F32G64, fem.FEM_BF16G64, fem.FEM_F16G64)


def kernel_family(op: str, N: int, epb: int, prec: int = fem.FEM_F64) -> str:
    """The kernel an apply runs with `epb` elements per workgroup (the
    library's dispatch): line-per-lane kernels with one element per
    workgroup (BP1.0, BP3.0 at every degree, BP3.5 from Nq = 9), the column
    kernels otherwise; BP3.0 in FP64 arithmetic at Nq = 11 and from Nq = 13
    runs the two-volume line kernel."""
    if op == "BP10":
        return "bp10t" if epb == 1 else "bp10"
    if op == "BP35":
        return "bp35t" if epb == 1 and N + 1 >= 9 else "bp35"
    if epb != 1:
        return "bp30"
    return "bp30t2" if prec in _F64_FIELDS and N + 1 >= 11 else "bp30t"


def lds_values(family: str, N: int) -> tuple[int, int]:
    """(values read, values written) in LDS per element by each kernel's
    schedule (s_r, s_w of the Empirical performance model section, eq.
    sharedRoof, in values of the compute type; q = Nq, g = Ng).  Uniform
    table reads (the same address on every lane) are not counted.

    * bp35 (lane per GLL column): u staged (q^3 writes); each point's r- and
      s-derivative read a row and a column (2 q^4), wr and ws staged (2 q^3),
      the transposes read a row and a column per point again (2 q^4).
    * bp35t (lane per line): u in, r-derivative out, s-derivative in place,
      metric step on QR and QS, two transposes in place, the final column
      sum: 8 q^3 reads, 7 q^3 writes.
    * bp10t (lane per line): every direction turned once through LDS (t- and
      s-interpolation, r-direction in place, s- and t-projection) plus the
      staged scaled Jacobians: 2 g q^2 + 2 g^2 q + g^3 reads and writes each.
    * bp10 (lane per output): r- and s-interpolation and s- and r-projection
      each read a whole line per output: 2 g q^3 + 2 g^2 q^2 reads;
      q^3 + 2 g q^2 + g^2 q writes.
    * bp30t (lane per line): the BP1.0 turns at both ends, the r-, s- and
      t-work on the Gauss grid (two derivatives out, metric step, two
      transposes, the r-transpose reading three volumes): 2 g q^2 + 2 g^2 q
      + 9 g^3 reads, 2 g q^2 + 2 g^2 q + 7 g^3 writes.
    * bp30t2 (the same with two volumes): u~ and its r-derivative written
      together, the metric lane's u~ column read once, the s-derivative in
      place, the t-term added to the s-term once: 2 g q^2 + 2 g^2 q + 8 g^3
      reads, 2 g q^2 + 2 g^2 q + 7 g^3 writes.
    * bp30 (lane per Gauss column): whole-line reads per output in the r- and
      s-interpolation and projection (2 g q^3 + 2 g^2 q^2) and in the
      gradient and its transpose (4 g^4); q^3 + 2 g q^2 + g^2 q + 3 g^3 writes.
    """
    q, g = N + 1, N + 2
    if family == "bp35":
        return 4 * q ** 4, 3 * q ** 3
    if family == "bp35t":
        return 8 * q ** 3, 7 * q ** 3
    if family == "bp10t":
        v = 2 * g * q * q + 2 * g * g * q + g ** 3
        return v, v
    if family == "bp10":
        return 2 * g * q ** 3 + 2 * g * g * q * q, q ** 3 + 2 * g * q * q + g * g * q
    if family == "bp30t":
        return 2 * g * q * q + 2 * g * g * q + 9 * g ** 3, 2 * g * q * q + 2 * g * g * q + 7 * g ** 3
    if family == "bp30t2":
        return 2 * g * q * q + 2 * g * g * q + 8 * g ** 3, 2 * g * q * q + 2 * g * g * q + 7 * g ** 3
    if family == "bp30":
        return 2 * g * q ** 3 + 2 * g * g * q * q + 4 * g ** 4, q ** 3 + 2 * g * q * q + g * g * q + 3 * g ** 3
    raise ValueError(family)


def lds_bytes(op: str, N: int, E: int, prec: int, epb: int) -> int:
    """LDS bytes (read + written) of one apply: values of the compute type
    (FP64 with FP64 fields, FP32 otherwise)."""
    r, w = lds_values(kernel_family(op, N, epb, prec), N)
    return E * (r + w) * (8 if prec in _F64_FIELDS else 4)


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


# persistent grid sizes tried for the column kernels: 4, 8 and 16 workgroups
# per CU of the 256, and uncapped (one workgroup per element group)
GRID_CAPS = (0, 1024, 2048, 4096)


def autotune(X: np.ndarray, ops=("BP10", "BP35", "BP30"), Ns=range(1, 16), precs=(fem.FEM_F64,),
             reps: int = 10, h: float | None = None, log=None, seed: int = 0,
             grid_caps=GRID_CAPS) -> list[dict]:
    """Time every supported packing of each (op, N, prec) on the mesh X, and
    for the column kernels every persistent grid size of `grid_caps`; returns
    one record per configuration with the fastest (packing, grid cap)."""
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
                        # the column kernels loop over element groups, so a
                        # capped grid makes them persistent; the line kernels
                        # only split their launch, so they run uncapped
                        caps = grid_caps if kernel_family(op, N, epb, prec) in ("bp10", "bp35", "bp30") else (0,)
                        for cap in caps:
                            fem.fem_tune_set(opid, N, prec, epb, cap)
                            timings[(epb, cap)] = _time(call, reps, stream)
                finally:
                    fem.fem_tune_set(opid, N, prec, 0, 0)
                (best, best_cap) = min(timings, key=timings.get)
                ms = timings[(best, best_cap)]
                # a cap is kept only where it beats the uncapped grid of the
                # same packing by more than 2%
                if best_cap and timings[(best, 0)] <= 1.02 * ms:
                    best_cap, ms = 0, timings[(best, 0)]
                nbytes = alg_bytes(op, N, E, prec)
                rec = dict(op=op, N=N, prec=prec, E=E, epb=best, grid_cap=best_cap, ms=ms,
                           gbs=nbytes / (ms * 1e-3) / 1e9, gdofs=E * dev.np / (ms * 1e-3) / 1e9,
                           tflops=alg_flops(op, N, E) / (ms * 1e-3) / 1e12,
                           all_ms={f"{k[0]}/{k[1]}": v for k, v in timings.items()})
                out.append(rec)
                if log:
                    log(f"tune {op} N={N} prec={prec}: epb {best} cap {best_cap} {ms:.4f} ms {rec['gbs']:.0f} GB/s "
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

"""Reduced-precision storage against the oracle.

A narrow-storage apply computes the operator of the rounded inputs: u, G and
wJ as stored (FP32, BF16, or FP16 times a power-of-two scale).  The oracle
applies its FP64 operator to the same inputs, rounded by its own code
(oracle/storage.py, from the formats' definitions), and the GPU result is
compared with that, element by element:

* modes with FP64 fields and FP64 arithmetic (F32G64, BF16G64, F16G64): the
  FP64 bar, relative L2 <= 1e-12 and per element <= 1e-11 of the element's
  largest output;
* modes with FP32 arithmetic (F32, BF16, F16, BF16G, F16G): the FP32
  arithmetic is then the only difference.  A priori an output passes through
  at most seven one-direction sums of at most 17 terms (BP3.0 at N = 15), so
  its rounding error is at most about 7 * 17 * 2^-24 = 7e-6 of the sum of the
  absolute terms.  Measured over every mode, operator and degree here (the
  table FEM_RECORD_DIR receives, kept in profiles/): at most 2.8e-7 relative
  L2 and 7.1e-7 per element, so the bound is about three times that:
  relative L2 <= 8e-7, per element <= 2e-6.  A result rounded once more than
  it should be, or scaled wrongly, exceeds it.

The error of each result against the FP64 oracle on the *unrounded* inputs --
the error the storage format costs -- is recorded per (mode, operator, N).
With FEM_RECORD_DIR set, the table is written there as
reduced_precision_errors.md (and .json).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import storage
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# mode: (field storage, geometry storage, arithmetic)
MODES = {1: ("f32", "f32", "f32"), 2: ("bf16", "bf16", "f32"), 3: ("f16", "f16", "f32"),
         4: ("f32", "bf16", "f32"), 5: ("f32", "f16", "f32"),
         6: ("f64", "f32", "f64"), 7: ("f64", "bf16", "f64"), 8: ("f64", "f16", "f64")}
MODE_NAMES = {1: "F32", 2: "BF16", 3: "F16", 4: "BF16G", 5: "F16G", 6: "F32G64", 7: "BF16G64", 8: "F16G64"}
BAR = {"f64": (1e-12, 1e-11), "f32": (8e-7, 2e-6)}
E = 64
ROWS = []


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh, FIELD_DTYPE
    fem.lib()
    yield fem, DeviceMesh, FIELD_DTYPE
    rec = os.environ.get("FEM_RECORD_DIR")
    if rec and ROWS:
        os.makedirs(rec, exist_ok=True)
        with open(os.path.join(rec, "reduced_precision_errors.json"), "w") as f:
            json.dump(ROWS, f, indent=1)
        lines = ["| mode | u / G storage | arithmetic | op | N | vs FP64 oracle (GPU) | vs FP64 oracle "
                 "(oracle on rounded inputs) | GPU vs oracle on rounded inputs |",
                 "|---|---|---|---|---|---|---|---|"]
        for r in ROWS:
            lines.append(f"| {r['mode']} | {r['u']} / {r['G']} | {r['arith']} | {r['op']} | {r['N']} | "
                         f"{r['err_exact']:.2e} | {r['err_pred']:.2e} | {r['err_rounded']:.2e} |")
        with open(os.path.join(rec, "reduced_precision_errors.md"), "w") as f:
            f.write("\n".join(lines) + "\n")


_ORA = {}


def oracle_geometry(N):
    if N not in _ORA:
        n = 4
        X = workloads.element_vertices(n, E=E)
        _ORA[N] = (X, oracle.geometry(N, X, "gll"), oracle.geometry(N, X, "gl"))
    return _ORA[N]


def oracle_apply(op, N, geo_gll, geo_gl, u, fmt_g, sG, swJ):
    if op == "BP10":
        return oracle.bp10(N, storage.stored(geo_gl[1], fmt_g, swJ), u)
    if op == "BP35":
        return oracle.bp35(N, storage.stored(geo_gll[0], fmt_g, sG), u)
    return oracle.bp30(N, storage.stored(geo_gl[0], fmt_g, sG), u)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", sorted(MODES))
@pytest.mark.parametrize("op", ["BP10", "BP35", "BP30"])
# N = 2 and 14 cover the low-degree column-kernel loads and the BP1.0 line
# kernel's wJ rows at Ng = 16
@pytest.mark.parametrize("N", [1, 2, 3, 7, 11, 14, 15])
def test_reduced_precision_parity(ctx, prec, op, N):
    fem, DeviceMesh, FIELD_DTYPE = ctx
    fmt_u, fmt_g, arith = MODES[prec]
    X, geo_gll, geo_gl = oracle_geometry(N)
    dev = DeviceMesh(N, X, h=1.0 / 4)
    sG, swJ = dev.geo_scale(prec, "G"), dev.geo_scale(prec, "wJ")
    u = workloads.field(E, N + 1, seed=21 + N)
    ur = storage.stored(u, fmt_u)                      # exactly representable in the storage type
    ut = torch.from_numpy(ur).cuda().to(FIELD_DTYPE[prec])
    assert torch.equal(ut.to(torch.float64).cpu(), torch.from_numpy(ur))
    if op == "BP10":
        y = dev.mass(ut, prec=prec)
    elif op == "BP35":
        y = dev.stiff35(ut, prec=prec)
    else:
        y = dev.stiff30(ut, prec=prec)
    torch.cuda.synchronize()
    assert y.dtype == (torch.float64 if arith == "f64" else torch.float32)
    yg = y.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(yg))
    ref_r = oracle_apply(op, N, geo_gll, geo_gl, ur, fmt_g, sG, swJ)
    ref_x = oracle_apply(op, N, geo_gll, geo_gl, u, "f64", 1.0, 1.0)
    e_r = rel(yg, ref_r)
    worst = float(np.max(np.abs(yg - ref_r).max(axis=1) / np.abs(ref_r).max(axis=1)))
    row = dict(mode=MODE_NAMES[prec], u=fmt_u, G=fmt_g, arith=arith, op=op, N=N, err_rounded=e_r,
               err_rounded_elem=worst, err_exact=rel(yg, ref_x), err_pred=rel(ref_r, ref_x))
    ROWS.append(row)
    print(row)
    bar, per = BAR[arith]
    assert e_r <= bar and worst <= per, row
    # the error against the FP64 operator is the storage error the oracle predicts
    assert abs(row["err_exact"] - row["err_pred"]) <= bar + 1e-3 * row["err_pred"], row

"""BP1.0's persistent line kernel (FP32 or 16-bit fields at Nq = 9..11,
FP64 fields with narrow wJ at Nq = 10..11): each workgroup walks the
elements e, e + G, ... with the next element's u and wJ requested before it
works on the current one.  With a grid capped at 1, 3 or 5 workgroups
(E = 64: ragged for 3 and 5) every workgroup walks many elements; the result
must equal the default grid's bit for bit (each element's arithmetic does
not depend on the grid), with beta = 0 and with beta != 0, and the default
grid must match the oracle on the rounded inputs (the bar of the
reduced-precision tests).  N = 6 and 7 (the one-shot kernel, whose capped
grid is split over launches) are controls.  The CG at N = 9, whose mass
apply takes the tuned grid, must give the same iterates with a capped BP1.0
grid as with the default one.
"""
import numpy as np
import pytest

import oracle
from oracle import storage
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = 64
# mode: (field storage, geometry storage, arithmetic)
MODES = {0: ("f64", "f64", "f64"), 1: ("f32", "f32", "f32"), 2: ("bf16", "bf16", "f32"),
         4: ("f32", "bf16", "f32"), 7: ("f64", "bf16", "f64")}
BAR = {"f64": (1e-12, 1e-11), "f32": (8e-7, 2e-6)}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh, FIELD_DTYPE
    fem.lib()
    return fem, DeviceMesh, FIELD_DTYPE


@pytest.mark.parametrize("prec", sorted(MODES))
@pytest.mark.parametrize("N", [6, 7, 8, 9, 10])
def test_capped_grid_same_bits_and_oracle(ctx, prec, N):
    fem, DeviceMesh, FIELD_DTYPE = ctx
    fmt_u, fmt_g, arith = MODES[prec]
    X = workloads.element_vertices(4, E=E)
    dev = DeviceMesh(N, X, h=1.0 / 4)
    u = storage.stored(workloads.field(E, N + 1, seed=40 + N), fmt_u)
    ut = torch.from_numpy(u).cuda().to(FIELD_DTYPE[prec])
    y0 = workloads.field(E, N + 1, seed=60 + N)
    ydt = torch.float64 if arith == "f64" else torch.float32
    ref = dev.mass(ut, prec=prec).clone()
    ref_b = dev.mass(ut, torch.from_numpy(y0).cuda().to(ydt), beta=0.5, prec=prec).clone()
    try:
        for cap in (1, 3, 5):
            fem.fem_tune_set(0, N, prec, 1, cap)
            y = dev.mass(ut, prec=prec)
            yb = dev.mass(ut, torch.from_numpy(y0).cuda().to(ydt), beta=0.5, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (N, prec, cap)
            assert torch.equal(yb, ref_b), (N, prec, cap, "beta")
    finally:
        fem.fem_tune_set(0, N, prec, 0, 0)
    geo_gl = oracle.geometry(N, X, "gl")
    want = oracle.bp10(N, storage.stored(geo_gl[1], fmt_g, dev.geo_scale(prec, "wJ")), u)
    got = ref.cpu().numpy().astype(np.float64)
    bar, per = BAR[arith]
    e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    worst = float(np.max(np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)))
    assert e <= bar and worst <= per, (N, prec, e, worst)
    got_b = ref_b.cpu().numpy().astype(np.float64)
    want_b = want + 0.5 * storage.stored(y0, "f64" if arith == "f64" else "f32")
    assert float(np.linalg.norm(got_b - want_b) / np.linalg.norm(want_b)) <= bar, (N, prec, "beta")


@pytest.mark.parametrize("mode,inner", [(1, 7), (2, 4)])
def test_cg_with_capped_mass_grid(ctx, mode, inner):
    """CG with BF16 geometry (FP64 vectors, mode 1) and iterative refinement
    (FP32 inner CG, mode 2) at N = 9: a BP1.0 grid of 3 workgroups gives the
    same iterates and residuals as the default grid."""
    fem, DeviceMesh, _ = ctx
    N = 9
    X = workloads.element_vertices(4, E=E)
    dev = DeviceMesh(N, X, h=1.0 / 4)
    b = torch.from_numpy(workloads.field(E, N + 1, seed=77)).cuda()
    runs = []
    for cap in (0, 3):
        try:
            fem.fem_tune_set(0, N, inner, 1, cap)
            x = torch.zeros_like(b)
            rep = dev.cg_solve(b, x, lam=2.0, mode=mode, inner_prec=inner, rtol=1e-9, max_iters=2000)
            torch.cuda.synchronize()
            runs.append((rep, x.clone()))
        finally:
            fem.fem_tune_set(0, N, inner, 0, 0)
    (r0, x0), (r1, x1) = runs
    assert r0["status"] == fem.FEM_OK and r0["rel_res"] <= 1e-9, r0
    assert r0["iters"] == r1["iters"] and r0["rel_res"] == r1["rel_res"], (r0, r1)
    assert torch.equal(x0, x1)

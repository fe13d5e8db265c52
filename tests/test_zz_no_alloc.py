"""fem_cg_solve_noalloc (the CG solve in the library's own device array)
against fem_cg_solve (the same solve in a caller-provided workspace).

Both run the same kernels in the same order on the same inputs, so the
iterates, reports and solutions must agree to the FP64 bar (relative L2
<= 1e-12; in practice bit for bit).  Two calls in a row, the second on a
smaller mesh, check that a call does not depend on what the previous one left
in the shared array.  A solve whose workspace exceeds the array is refused
before anything is enqueued.  The operator is the CG workload's,
S(BP3.5) + lambda M(BP1.0) at N = 7 on the first elements of the 64^3 mesh;
the oracle re-evaluates the residual of the no-allocation solution.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.cg import true_relative_residual
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 7
NGRID = 64


def problem(E):
    from paper_1711_00903_amd.mesh import DeviceMesh
    X = workloads.element_vertices(NGRID, E=E)
    noise = workloads.rhs_noise(E, N + 1)
    dev = DeviceMesh(N, X, h=1.0 / NGRID)
    xyz = dev.node_coords()
    b = (torch.sin(math.pi * xyz[..., 0]) * torch.sin(math.pi * xyz[..., 1]) *
         torch.sin(math.pi * xyz[..., 2]) + 1e-3 * torch.from_numpy(noise).cuda()).contiguous()
    return X, noise, dev, b


def oracle_residual(X, noise, x, lam):
    pb = oracle.Problem(N, X)
    xo = oracle.node_coords(N, X, "gll")
    bo = np.sin(np.pi * xo[..., 0]) * np.sin(np.pi * xo[..., 1]) * np.sin(np.pi * xo[..., 2]) + 1e-3 * noise
    return true_relative_residual(lambda v: pb.cg_operator(v, lam), bo, x)


# (elements, lambda, mode, inner storage): the second call is smaller
CALLS = [(512, 1.0, 0, 0), (96, 4096.0, 1, 7)]


def test_noalloc_matches_workspace_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem
    fem.lib()
    for E, lam, mode, inner in CALLS:
        X, noise, dev, b = problem(E)
        rtol = 1e-9
        print(f"noalloc: E={E} lambda={lam} mode={mode} inner={inner}", flush=True)
        x_ref = torch.zeros_like(b)
        rep_ref = dev.cg_solve(b, x_ref, lam=lam, mode=mode, inner_prec=inner, rtol=rtol)
        x = torch.full_like(b, 0.0)
        rep = dev.cg_solve(b, x, lam=lam, mode=mode, inner_prec=inner, rtol=rtol, noalloc=True)
        torch.cuda.synchronize()
        print(f"noalloc: workspace {rep_ref}, no allocation {rep}", flush=True)
        assert rep["status"] == fem.FEM_OK and rep_ref["status"] == fem.FEM_OK
        for k in ("iters", "reliable_updates", "hi_matvecs"):
            assert rep[k] == rep_ref[k], k
        xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
        err = np.linalg.norm(xn - xr) / np.linalg.norm(xr)
        assert err <= 1e-12, err
        assert abs(rep["rel_res"] - rep_ref["rel_res"]) <= 1e-12 * rep_ref["rel_res"] + 1e-300
        res = oracle_residual(X, noise, xn, lam)
        assert res <= 1.1 * rtol, res
        del dev, b, x, x_ref
        torch.cuda.empty_cache()


def test_noalloc_refuses_oversize():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh
    fem.lib()
    # 4096 elements at N = 7 need more than the array (2.1M DOFs x ~48 B)
    X = workloads.element_vertices(16)
    dev = DeviceMesh(N, X, h=1.0 / 16)
    op, opt, _ = dev.cg_structs(1.0)
    assert fem.fem_cg_workspace_bytes(op, opt) > fem.FEM_CG_NOALLOC_BYTES
    b = torch.ones((X.shape[0], (N + 1) ** 3), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(fem.FemError) as ei:
        fem.fem_cg_solve_noalloc(op, opt, b, x)
    assert ei.value.status == fem.FEM_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0

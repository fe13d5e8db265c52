"""The assembled operator Z^T (S + lambda M) Z, its Jacobi diagonal and
Jacobi-PCG, through the C ABI, against the oracle (oracle/assembly.py).

* gather and scatter are index work with sums in one fixed order (ascending
  local node): bit for bit equal to the oracle's;
* the assembled operator and its diagonal: relative L2 <= 1e-12;
* PCG: the oracle's own FP64 evaluation of ||b - A x|| / ||b|| meets the
  tolerance (within 10%), and the iteration count is that of the oracle's
  textbook PCG to within 10%.
Meshes: perturbed structured grids, whole (n^3 elements) and partial (the
first E elements, so the boundary is ragged), at several degrees.
"""
import numpy as np
import pytest

import oracle
from oracle import assembly
from oracle.cg import pcg, true_relative_residual
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem as f
    f.lib()
    return f


def mesh(N, n, E=None):
    from paper_1711_00903_amd.mesh import DeviceMesh
    X = workloads.element_vertices(n, E=E)
    gids, ng = workloads.global_numbering(n, N, E=X.shape[0])
    dev = DeviceMesh(N, X, h=1.0 / n)
    dev.set_assembly(gids, ng)
    return X, gids, ng, dev


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N,n,E", [(1, 4, None), (3, 3, 20), (7, 3, None), (12, 2, 7)])
def test_gather_scatter_bitwise(fem, N, n, E):
    X, gids, ng, dev = mesh(N, n, E)
    nl = gids.size
    ug = np.random.default_rng(N).uniform(-1, 1, ng)
    ul = torch.empty(nl, dtype=torch.float64, device="cuda")
    fem.fem_gather(nl, ng, dev._gather, torch.from_numpy(ug).cuda(), ul)
    vl = np.random.default_rng(N + 1).uniform(-1, 1, nl)
    vg = torch.empty(ng, dtype=torch.float64, device="cuda")
    fem.fem_scatter(nl, ng, dev._offsets, dev._locals, torch.from_numpy(vl).cuda(), vg)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ul.cpu().numpy(), assembly.gather(ug, gids).ravel())
    np.testing.assert_array_equal(vg.cpu().numpy(), assembly.scatter(vl.reshape(gids.shape), gids, ng))


@pytest.mark.parametrize("lam", [0.0, 1.0])
@pytest.mark.parametrize("N,n,E", [(1, 4, None), (2, 3, 20), (5, 3, None), (7, 4, 50), (11, 2, None),
                                   (15, 2, 5)])
def test_assembled_apply_and_diagonal(fem, N, n, E, lam):
    X, gids, ng, dev = mesh(N, n, E)
    ug = np.random.default_rng(3 + N).uniform(-1, 1, ng)
    yg = dev.assembled_apply(torch.from_numpy(ug).cuda(), lam=lam).cpu().numpy()
    pb = oracle.Problem(N, X)
    ref = assembly.assembled_apply(lambda u: pb.cg_operator(u, lam), gids, ng, ug)
    assert rel(yg, ref) <= 1e-12, rel(yg, ref)
    d = dev.assembled_diagonal(lam=lam).cpu().numpy()
    dl = assembly.stiff35_diag(N, pb.G_gll())
    if lam:
        dl = dl + lam * assembly.mass_diag(N, pb.wJ_gl())
    dref = assembly.scatter(dl, gids, ng)
    assert rel(d, dref) <= 1e-12, rel(d, dref)


def test_assembled_apply_repeatable(fem):
    X, gids, ng, dev = mesh(7, 4)
    ug = torch.from_numpy(np.random.default_rng(9).uniform(-1, 1, ng)).cuda()
    a = dev.assembled_apply(ug).clone()
    b = dev.assembled_apply(ug).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def rhs(X, gids, ng, N):
    """b = sin(pi x) sin(pi y) sin(pi z) + 1e-3 U[-1,1] at each global node
    (coordinates of the node's first local copy)."""
    xyz = oracle.node_coords(N, X, "gll").reshape(-1, 3)
    first = np.full(ng, -1, dtype=np.int64)
    flat = gids.ravel()
    first[flat[::-1]] = np.arange(flat.size)[::-1]
    xg = xyz[first]
    return np.sin(np.pi * xg[:, 0]) * np.sin(np.pi * xg[:, 1]) * np.sin(np.pi * xg[:, 2]) + \
        1e-3 * workloads.global_noise(ng)


@pytest.mark.parametrize("lam", [1.0, 4096.0])
def test_pcg_against_oracle(fem, lam):
    """N = 7 on the first 512 elements of the 64^3 mesh (h = 1/64)."""
    N = 7
    X, gids, ng, dev = mesh(N, 64, 512)
    b = rhs(X, gids, ng, N)
    rtol = 1e-8
    pb = oracle.Problem(N, X)
    A = lambda v: assembly.assembled_apply(lambda u: pb.cg_operator(u, lam), gids, ng, v)
    dl = assembly.stiff35_diag(N, pb.G_gll()) + lam * assembly.mass_diag(N, pb.wJ_gl())
    dg = assembly.scatter(dl, gids, ng)
    bt = torch.from_numpy(b).cuda()
    its = {}
    for jacobi in (True, False):
        x = torch.zeros_like(bt)
        rep = dev.pcg_solve(bt, x, lam=lam, jacobi=jacobi, rtol=rtol, history=64)
        torch.cuda.synchronize()
        print(f"lambda={lam} jacobi={jacobi}: {rep}", flush=True)
        assert rep["status"] == fem.FEM_OK and rep["rel_res"] <= rtol
        res = true_relative_residual(A, b, x.cpu().numpy())
        assert res <= 1.1 * rtol, res
        _, it_o, _ = pcg(A, b, (lambda r: r / dg) if jacobi else (lambda r: r.copy()), rtol=rtol)
        assert abs(rep["iters"] - it_o) <= max(3, 0.1 * it_o), (rep["iters"], it_o)
        its[jacobi] = rep["iters"]
    assert its[True] < its[False]

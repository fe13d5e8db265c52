"""Ragged batches (fem_batch_apply) and their graph capture against the oracle.

Meshes of different degrees, sizes and operators in one batch; each output is
compared with the oracle (FP64 to 1e-12 relative, FP32 within the storage
error bound).  Graph replays are checked bit for bit against the eager batch,
with eager work and synchronisation between the replays.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MESHES = [("BP35", 7, 27), ("BP10", 3, 64), ("BP30", 5, 20), ("BP35", 2, 100), ("BP30", 1, 7),
          ("BP10", 11, 8), ("BP35", 14, 5), ("BP30", 9, 12), ("BP10", 6, 30), ("BP30", 7, 9)]


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem
    from paper_1711_00903_amd.mesh import DeviceMesh
    fem.lib()
    items = []
    for m, (op, N, E) in enumerate(MESHES):
        n = 1
        while n ** 3 < E:
            n += 1
        X = workloads.element_vertices(n, E=E, seed=workloads.SEED_MESH + m)
        u = workloads.field(E, N + 1, seed=workloads.SEED_FIELD + m)
        dev = DeviceMesh(N, X, h=1.0 / n)
        pb = oracle.Problem(N, X)
        ref = {"BP10": pb.mass, "BP35": pb.stiff35, "BP30": pb.stiff30}[op](u)
        items.append(dict(op=op, N=N, E=E, dev=dev, u=u, ref=ref))
    return fem, items


def make(fem, items, prec):
    from paper_1711_00903_amd.mesh import FIELD_DTYPE, out_dtype
    descs, outs = [], []
    for it in items:
        ut = torch.from_numpy(it["u"]).cuda().to(FIELD_DTYPE[prec])
        yt = torch.zeros(it["u"].shape, dtype=out_dtype(prec), device="cuda")
        it.setdefault("keep", []).append(ut)
        descs.append(it["dev"].desc(it["op"], ut, yt, prec=prec))
        outs.append(yt)
    return descs, outs


def rel(y, ref):
    return np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (7, 6e-2)])
def test_batch_matches_oracle(batch, prec, tol):
    fem, items = batch
    descs, outs = make(fem, items, prec)
    fem.fem_batch_apply(descs)
    torch.cuda.synchronize()
    for it, y in zip(items, outs):
        assert rel(y, it["ref"]) <= tol, (it["op"], it["N"], prec)


@pytest.mark.parametrize("lanes", [1, 4])
def test_graph_replays_match_eager(batch, lanes):
    fem, items = batch
    descs, outs = make(fem, items, 0)
    fem.fem_batch_apply(descs)
    torch.cuda.synchronize()
    eager = [y.clone() for y in outs]
    stream = torch.cuda.Stream()
    g = fem.BatchGraph(descs, lanes=lanes, stream=stream)
    for rep in range(3):
        for y in outs:
            y.zero_()                         # eager work between replays
        torch.cuda.synchronize()
        g.launch(stream=stream)
        stream.synchronize()
        for y, e in zip(outs, eager):
            assert torch.equal(y, e), rep
    g.destroy()


def test_bad_descriptor_enqueues_nothing(batch):
    fem, items = batch
    descs, outs = make(fem, items, 0)
    descs[3].N = 0
    with pytest.raises(fem.FemError) as ei:
        fem.fem_batch_apply(descs)
    assert ei.value.status == fem.FEM_ERR_ARG
    torch.cuda.synchronize()
    assert all(float(y.abs().max()) == 0.0 for y in outs)
    with pytest.raises(fem.FemError):
        fem.BatchGraph(descs, lanes=2, stream=torch.cuda.Stream())

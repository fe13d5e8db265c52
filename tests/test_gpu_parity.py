"""GPU parity: libfem's HIP kernels against the FP64 CPU oracle.

Both sides start from the same seeded vertices and fields (``workloads``) and
build their own tables and geometric factors.  FP64 bar (from the operators'
specification): relative L2 error <= 1e-12 per call, and per element
max |y_gpu - y_oracle| <= 1e-11 * max |y_oracle| of that element.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_L2 = 1e-12
PER_ELEM = 1e-11


@pytest.fixture(scope="module")
def fem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_00903_amd import fem as f
    f.lib()
    return f


@pytest.fixture(scope="module")
def DeviceMesh(fem):
    from paper_1711_00903_amd.mesh import DeviceMesh as DM
    return DM


def compare(y, ref, tag, rel=REL_L2, per=PER_ELEM):
    y = y.detach().cpu().numpy().astype(np.float64) if torch.is_tensor(y) else y
    assert y.shape == ref.shape, (tag, y.shape, ref.shape)
    assert np.all(np.isfinite(y)), tag
    nref = np.linalg.norm(ref)
    err = np.linalg.norm(y - ref) / nref if nref else np.linalg.norm(y)
    assert err <= rel, f"{tag}: rel-L2 {err:.3e}"
    if per is not None and ref.shape[0]:
        emax = np.abs(y - ref).max(axis=1)
        scale = np.abs(ref).max(axis=1)
        worst = np.max(emax / np.where(scale > 0, scale, 1.0))
        assert worst <= per, f"{tag}: per-element {worst:.3e}"
    return err


_CACHE = {}


def oracle_apply(op, N, X, u, lam=0.0):
    key = (op, N, X.shape[0], lam, u.shape, float(u.ravel()[:4].sum()) if u.size else 0.0)
    if key not in _CACHE:
        pb = oracle.Problem(N, X)
        _CACHE[key] = {"BP10": lambda: pb.mass(u),
                       "BP35": lambda: pb.stiff35(u, lam),
                       "BP30": lambda: pb.stiff30(u, lam)}[op]()
    return _CACHE[key]


def gpu_apply(dev, op, ut, lam=0.0, prec=0, y=None, beta=0.0):
    if op == "BP10":
        return dev.mass(ut, y=y, beta=beta, prec=prec)
    if op == "BP35":
        return dev.stiff35(ut, y=y, lam=lam, beta=beta, prec=prec)
    return dev.stiff30(ut, y=y, lam=lam, beta=beta, prec=prec)


def mesh_elems(E):
    n = 1
    while n ** 3 < E:
        n += 1
    return workloads.element_vertices(n, E=E), n


# ---------------------------------------------------------------- geometry

@pytest.mark.parametrize("N", [1, 2, 7, 15])
@pytest.mark.parametrize("quad", [0, 1])
def test_geometry_parity(fem, DeviceMesh, N, quad):
    X = workloads.element_vertices(3)
    dev = DeviceMesh(N, X, h=1 / 3)
    G, wJ = dev.geometry(quad)
    n = N + 1 + quad
    off = torch.from_numpy(fem.geo_layout_offsets(n, fem.fem_geo_vector_width(N, quad, 0))).cuda()
    G, wJ = G[:, :, off], wJ[:, off]          # back to the natural node order
    Go, wJo = oracle.geometry(N, X, "gll" if quad == 0 else "gl")
    compare(G.reshape(G.shape[0], -1), Go.reshape(Go.shape[0], -1), "G", rel=1e-14, per=1e-13)
    compare(wJ, wJo, "wJ", rel=1e-14, per=1e-13)
    xyz = dev.node_coords(quad).cpu().numpy()
    np.testing.assert_allclose(xyz, oracle.node_coords(N, X, "gll" if quad == 0 else "gl"),
                               rtol=0, atol=1e-15)


def test_geometry_flags_inverted_element(fem, DeviceMesh):
    X = workloads.element_vertices(2)
    X[3, [0, 1]] = X[3, [1, 0]]
    dev = DeviceMesh(3, X, h=0.5)
    with pytest.raises(fem.FemError) as ei:
        dev.geometry(1)
    assert ei.value.status == fem.FEM_ERR_GEOMETRY


# ---------------------------------------------------------------- operators, all degrees

def _epb_cases():
    from paper_1711_00903_amd import fem as f
    out = []
    for op in ("BP10", "BP35", "BP30"):
        for N in range(1, 16):
            try:
                f.lib()
                chs = f.fem_supported_epb(f.OP_NAMES[op], N, 0)
            except Exception:
                chs = [1]
            for c in chs:
                out.append((op, N, c))
    return out


@pytest.mark.parametrize("op,N,epb", _epb_cases())
def test_operator_parity_all_degrees(fem, DeviceMesh, op, N, epb):
    """Every degree and every supported packing, on a ragged 61-element mesh
    (several workgroups plus a partial last group) and on a single element."""
    opid = fem.OP_NAMES[op]
    fem.fem_tune_set(opid, N, 0, epb, 0)
    try:
        for E in (61, 1):
            X, n = mesh_elems(E)
            u = workloads.field(E, N + 1, seed=100 + N)
            dev = DeviceMesh(N, X, h=1.0 / n)
            y = gpu_apply(dev, op, torch.from_numpy(u).cuda())
            torch.cuda.synchronize()
            compare(y, oracle_apply(op, N, X, u), f"{op} N={N} epb={epb} E={E}")
    finally:
        fem.fem_tune_set(opid, N, 0, 0, 0)


@pytest.mark.parametrize("op", ["BP35", "BP30"])
@pytest.mark.parametrize("N", [2, 7, 11, 14])
def test_lambda_and_beta(fem, DeviceMesh, op, N):
    X, n = mesh_elems(40)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=5)
    y0 = workloads.field(E, N + 1, seed=6)
    lam, beta = 0.75, -0.5
    dev = DeviceMesh(N, X, h=1.0 / n)
    yt = torch.from_numpy(y0).cuda()
    gpu_apply(dev, op, torch.from_numpy(u).cuda(), lam=lam, y=yt, beta=beta)
    torch.cuda.synchronize()
    ref = oracle_apply(op, N, X, u, lam) + beta * y0
    compare(yt, ref, f"{op} lambda/beta")


def test_mass_beta(fem, DeviceMesh):
    N = 5
    X, n = mesh_elems(30)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=7)
    y0 = workloads.field(E, N + 1, seed=8)
    dev = DeviceMesh(N, X, h=1.0 / n)
    yt = torch.from_numpy(y0).cuda()
    dev.mass(torch.from_numpy(u).cuda(), y=yt, beta=2.0)
    torch.cuda.synchronize()
    compare(yt, oracle_apply("BP10", N, X, u) + 2.0 * y0, "mass beta")


# ---------------------------------------------------------------- determinism

@pytest.mark.parametrize("op", ["BP10", "BP35", "BP30"])
def test_repeatable_bitwise(fem, DeviceMesh, op):
    N = 7
    X, n = mesh_elems(300)
    u = torch.from_numpy(workloads.field(X.shape[0], N + 1, seed=9)).cuda()
    dev = DeviceMesh(N, X, h=1.0 / n)
    a = gpu_apply(dev, op, u).clone()
    b = gpu_apply(dev, op, u).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_grid_cap_persistent_loop(fem, DeviceMesh):
    """A capped grid walks the element groups in a loop: same result."""
    N = 7
    X, n = mesh_elems(500)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=12)
    dev = DeviceMesh(N, X, h=1.0 / n)
    ut = torch.from_numpy(u).cuda()
    # (BP1.0 with one element per workgroup is the one-wave kernel, which
    # splits a capped grid over several launches instead)
    for op, epb in (("BP10", 0), ("BP10", 1), ("BP35", 0), ("BP30", 0)):
        opid = fem.OP_NAMES[op]
        try:
            fem.fem_tune_set(opid, N, 0, epb, 7)
            y = gpu_apply(dev, op, ut)
            torch.cuda.synchronize()
            compare(y, oracle_apply(op, N, X, u), f"{op} epb={epb} capped grid")
        finally:
            fem.fem_tune_set(opid, N, 0, 0, 0)


def test_grid_cap_line_kernels_high_degree(fem, DeviceMesh):
    """The line-per-lane kernels at high degree (half tables in LDS) split a
    capped grid over several launches: same result, ragged last launch."""
    N = 12
    X, n = mesh_elems(60)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=13)
    dev = DeviceMesh(N, X, h=1.0 / n)
    ut = torch.from_numpy(u).cuda()
    for op in ("BP10", "BP35", "BP30"):
        opid = fem.OP_NAMES[op]
        try:
            fem.fem_tune_set(opid, N, 0, 1, 7)
            y = gpu_apply(dev, op, ut)
            torch.cuda.synchronize()
            compare(y, oracle_apply(op, N, X, u), f"{op} N={N} epb=1 capped grid")
        finally:
            fem.fem_tune_set(opid, N, 0, 0, 0)


@pytest.mark.parametrize("N", [1, 3, 7, 10, 15])
def test_vertex_geometry_stiffness(fem, DeviceMesh, N):
    """BP3.5 with the factors formed in the kernel from the vertices: the
    oracle's operator (factors from the same trilinear map), with lambda and
    beta, and the stored-factor kernel on the same input."""
    X, n = mesh_elems(30)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=21)
    y0 = workloads.field(E, N + 1, seed=22)
    dev = DeviceMesh(N, X, h=1.0 / n)
    ut = torch.from_numpy(u).cuda()
    y = dev.stiff35_vertices(ut)
    torch.cuda.synchronize()
    compare(y, oracle_apply("BP35", N, X, u), f"BP35 vertices N={N}")
    ys = dev.stiff35(ut)
    torch.cuda.synchronize()
    compare(y, ys.cpu().numpy(), f"BP35 vertices vs stored factors N={N}")
    lam, beta = 0.75, -0.5
    yt = torch.from_numpy(y0).cuda()
    dev.stiff35_vertices(ut, y=yt, lam=lam, beta=beta)
    torch.cuda.synchronize()
    compare(yt, oracle_apply("BP35", N, X, u, lam) + beta * y0, f"BP35 vertices lambda/beta N={N}")


@pytest.mark.parametrize("N", [1, 3, 7, 10, 15])
def test_vertex_geometry_dealiased(fem, DeviceMesh, N):
    """BP3.0 with the factors formed in the kernel from the vertices: the
    oracle's operator, with lambda and beta, and the stored-factor kernel."""
    X, n = mesh_elems(30)
    E = X.shape[0]
    u = workloads.field(E, N + 1, seed=23)
    y0 = workloads.field(E, N + 1, seed=24)
    dev = DeviceMesh(N, X, h=1.0 / n)
    ut = torch.from_numpy(u).cuda()
    y = dev.stiff30_vertices(ut)
    torch.cuda.synchronize()
    compare(y, oracle_apply("BP30", N, X, u), f"BP30 vertices N={N}")
    ys = dev.stiff30(ut)
    torch.cuda.synchronize()
    compare(y, ys.cpu().numpy(), f"BP30 vertices vs stored factors N={N}")
    lam, beta = 0.75, -0.5
    yt = torch.from_numpy(y0).cuda()
    dev.stiff30_vertices(ut, y=yt, lam=lam, beta=beta)
    torch.cuda.synchronize()
    compare(yt, oracle_apply("BP30", N, X, u, lam) + beta * y0, f"BP30 vertices lambda/beta N={N}")


# ---------------------------------------------------------------- full-size workloads

def test_full_size_bp35_n7_e32768(fem, DeviceMesh):
    """The benchmarked workload (32^3 elements, N = 7) in the launch
    configuration the benchmark times, compared element by element in full."""
    N, n = 7, 32
    X = workloads.element_vertices(n)
    E = X.shape[0]
    u = workloads.field(E, N + 1)
    dev = DeviceMesh(N, X, h=1.0 / n)
    y = dev.stiff35(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    oracle.set_threads(0)
    ref = oracle.Problem(N, X).stiff35(u)
    compare(y, ref, "BP3.5 N=7 E=32768")


def _sampled(E):
    idx = np.unique(np.concatenate([np.arange(0, E, 64), np.arange(1024),
                                    np.arange(E - 1024, E)]))
    return idx


@pytest.mark.parametrize("op", ["BP30", "BP35", "BP10"])
def test_full_size_n7_e262144_sampled(fem, DeviceMesh, op):
    """64^3 elements at N = 7 (the de-aliased workload and the sweep size),
    checked on every 64th element plus the first and last 1024."""
    N, n = 7, 64
    E = n ** 3
    V = workloads.grid_vertices(n)
    X = workloads.element_vertices(n, V=V)
    dev = DeviceMesh(N, X, h=1.0 / n)
    ut = torch.empty((E, (N + 1) ** 3), dtype=torch.float64, device="cuda")
    for start, blk in workloads.field_chunked(E, N + 1, chunk=1 << 15):
        ut[start:start + blk.shape[0]] = torch.from_numpy(blk).cuda()
    y = gpu_apply(dev, op, ut)
    torch.cuda.synchronize()
    idx = _sampled(E)
    ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
    del y, ut
    dev.drop_geometry()
    torch.cuda.empty_cache()
    us = workloads.field_rows(E, N + 1, idx, chunk=1 << 15)
    Xs = workloads.element_vertices_subset(n, idx, V=V)
    ref = oracle_apply(op, N, Xs, us)
    compare(ys, ref, f"{op} N=7 E=262144 sampled")


@pytest.mark.parametrize("op", ["BP10", "BP35", "BP30"])
def test_max_degree_full_mesh(fem, DeviceMesh, op):
    N = 15
    X, n = mesh_elems(125)
    u = workloads.field(X.shape[0], N + 1, seed=31)
    dev = DeviceMesh(N, X, h=1.0 / n)
    y = gpu_apply(dev, op, torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    compare(y, oracle_apply(op, N, X, u), f"{op} N=15")


# ---------------------------------------------------------------- misc device paths

def test_stream_copy(fem):
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (1 << 20,), dtype=torch.int32, device="cuda")
    for nbytes in (16, 4096, (1 << 22) - 48, 1 << 22):
        dst = torch.zeros_like(src)
        fem.fem_stream_copy(src, dst, nbytes)
        torch.cuda.synchronize()
        k = nbytes // 4
        assert torch.equal(dst[:k], src[:k]) and not torch.any(dst[k:] != 0)


def test_empty_and_misaligned(fem, DeviceMesh):
    N = 3
    X, n = mesh_elems(8)
    dev = DeviceMesh(N, X, h=0.5)
    G, _ = dev.geometry(0)
    u = torch.zeros(8 * 64 + 1, dtype=torch.float64, device="cuda")
    y = torch.zeros(8 * 64 + 1, dtype=torch.float64, device="cuda")
    fem.fem_stiff_collocated_apply(N, 0, dev.D1d, G, None, 0.0, u, y)
    with pytest.raises(fem.FemError) as ei:
        fem.fem_stiff_collocated_apply(N, 8, dev.D1d, G, None, 0.0, u[1:], y)
    assert ei.value.status == fem.FEM_ERR_ALIGN

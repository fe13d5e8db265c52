"""CPU-side checks of libfem: it loads, exports every symbol fem.h declares, and
its host logic (tables, tune table, argument validation) behaves.  No compute
call reaches a GPU here: every apply below is rejected during validation,
before anything is enqueued."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fem():
    from paper_1711_00903_amd import fem as f
    if not os.path.exists(f.LIB_PATH):
        pytest.skip("libfem.so not built")
    f.lib()
    return f


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "fem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(fem):
    import ctypes
    L = ctypes.CDLL(fem.LIB_PATH)
    syms = header_symbols()
    assert "fem_stiff_collocated_apply" in syms and len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) <= set(fem.symbols())


def test_status_strings(fem):
    assert fem.status_str(0) == "ok"
    for s in range(1, 9):
        assert fem.status_str(s) not in ("ok", "unknown status")
    assert fem.fem_max_degree() == 15


@pytest.mark.parametrize("N", range(1, 16))
def test_product_tables_match_oracle(fem, N):
    T = fem.fem_basis_tables(N)
    O = oracle.tables(N)
    np.testing.assert_allclose(T["r_gll"], O.rgll, atol=1e-15)
    np.testing.assert_allclose(T["w_gll"], O.wgll, rtol=1e-13)
    np.testing.assert_allclose(T["r_gl"], O.rgl, atol=1e-15)
    np.testing.assert_allclose(T["w_gl"], O.wgl, rtol=1e-13)
    np.testing.assert_allclose(T["I1d"], O.I, atol=1e-14)
    np.testing.assert_allclose(T["D1d"], O.D, atol=1e-13 * N * N)
    np.testing.assert_allclose(T["Dgl"], O.Dgl, atol=1e-13 * N * N)


def test_bad_degree(fem):
    for N in (0, 16, -1):
        with pytest.raises(fem.FemError):
            fem.fem_basis_tables(N)


def test_tune_table(fem):
    for op in range(3):
        for N in range(1, 16):
            ch = fem.fem_supported_epb(op, N, fem.FEM_F64)
            assert ch and ch[0] == 1
            for c in ch:
                th, lds = fem.fem_kernel_info(op, N, fem.FEM_F64, c)
                assert th % 64 == 0 and 64 <= th <= 512
                assert 0 < lds <= 160 * 1024
    # BP1.0 with one element per workgroup runs the line-per-lane kernel (one
    # lane per GLL column: one wave up to N = 7); BP3.0 one lane per Gauss column
    for N in range(1, 16):
        th, _ = fem.fem_kernel_info(fem.FEM_OP_BP10, N, fem.FEM_F64, 1)
        assert th == (N + 1) ** 2 + (-(N + 1) ** 2) % 64, (N, th)
        th, _ = fem.fem_kernel_info(fem.FEM_OP_BP30, N, fem.FEM_F64, 1)
        assert th == (N + 2) ** 2 + (-(N + 2) ** 2) % 64, (N, th)
    fem.fem_tune_set(fem.FEM_OP_BP35, 7, fem.FEM_F64, 2, 1024)
    assert fem.fem_tune_get(fem.FEM_OP_BP35, 7, fem.FEM_F64) == (2, 1024)
    fem.fem_tune_set(fem.FEM_OP_BP35, 7, fem.FEM_F64, 0, 0)
    assert fem.fem_tune_get(fem.FEM_OP_BP35, 7, fem.FEM_F64)[1] == 0
    with pytest.raises(fem.FemError) as ei:
        fem.fem_tune_set(fem.FEM_OP_BP35, 7, fem.FEM_F64, 3 * 64 + 1, 0)
    assert ei.value.status == fem.FEM_ERR_UNSUPPORTED
    with pytest.raises(fem.FemError):
        fem.fem_tune_set(5, 7, 0, 0, 0)


def test_validation_rejects_before_enqueue(fem):
    """Each of these fails argument validation; none touches the device."""
    bad = 0x1000   # a fake, aligned device address: never dereferenced
    cases = [
        (lambda: fem.fem_stiff_collocated_apply(0, 4, bad, bad, None, 0.0, bad, bad + 4096, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_apply(16, 4, bad, bad, None, 0.0, bad, bad + 4096, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_apply(7, -1, bad, bad, None, 0.0, bad, bad + 4096, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_apply(7, 4, bad, bad, None, 1.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ARG),   # lambda != 0 needs wJ
        (lambda: fem.fem_stiff_collocated_apply(7, 4, bad, bad, None, 0.0, bad, bad, stream=0),
         fem.FEM_ERR_ARG),   # u == y
        (lambda: fem.fem_stiff_collocated_apply(7, 4, bad, bad, None, 0.0, bad + 8, 1 << 40, stream=0),
         fem.FEM_ERR_ALIGN),
        (lambda: fem.fem_stiff_collocated_apply(7, 4, bad, bad, None, 0.0, bad, 1 << 40, prec=12,
                                                stream=0), fem.FEM_ERR_UNSUPPORTED),
        (lambda: fem.fem_stiff_collocated_apply(7, 4, bad, bad, None, 0.0, bad, 1 << 40, prec=3,
                                                geo_scale=0.0, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_mass_apply(7, 4, None, bad, bad, 1 << 40, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_mass_apply(3, 1 << 31, bad, bad, bad, 1 << 40, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_dealiased_apply(7, 4, bad, None, bad, None, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_geometric_factors(7, 4, 2, bad, bad, bad, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_geometric_factors(7, 4, 0, bad, None, None, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_vertex_apply(0, 4, bad, bad, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_vertex_apply(7, 4, bad, None, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_collocated_vertex_apply(7, 4, bad, bad, 0.0, bad, bad, stream=0),
         fem.FEM_ERR_ARG),   # u == y
        (lambda: fem.fem_stiff_collocated_vertex_apply(7, 4, bad, bad + 8, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ALIGN),
        (lambda: fem.fem_stiff_dealiased_vertex_apply(16, 4, bad, bad, bad, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ARG),
        (lambda: fem.fem_stiff_dealiased_vertex_apply(7, 4, bad, bad, bad + 8, 0.0, bad, 1 << 40, stream=0),
         fem.FEM_ERR_ALIGN),
        (lambda: fem.fem_stream_copy(bad, 1 << 40, 17, stream=0), fem.FEM_ERR_ARG),
        (lambda: fem.fem_stream_copy(bad, bad + 16, 64, stream=0), fem.FEM_ERR_ARG),
    ]
    for i, (f, st) in enumerate(cases):
        with pytest.raises(fem.FemError) as ei:
            f()
        assert ei.value.status == st, (i, ei.value.status, st)


def test_empty_calls_are_noops(fem):
    fem.fem_stiff_collocated_apply(7, 0, None, None, None, 0.0, None, None, stream=0)
    fem.fem_mass_apply(3, 0, None, None, None, None, stream=0)
    fem.fem_stiff_dealiased_apply(5, 0, None, None, None, None, 0.0, None, None, stream=0)
    fem.fem_stream_copy(None, None, 0, stream=0)
    fem.fem_stiff_collocated_vertex_apply(7, 0, None, None, 0.0, None, None, stream=0)


def test_cg_struct_layout_matches_header(fem, tmp_path):
    """The ctypes structs of the binding have the header's field offsets."""
    import ctypes
    import subprocess
    fields = {"fem_cg_operator": ("CgOperator", ["N", "E", "I1d", "D1d", "G", "wJ", "lambda", "inner_prec",
                                                 "G_lo", "wJ_lo", "geo_scale_G", "geo_scale_wJ"]),
              "fem_cg_options": ("CgOptions", ["mode", "rtol", "max_iters", "delta", "check_every",
                                               "fusion", "history", "history_len"]),
              "fem_cg_report": ("CgReport", ["status", "iters", "reliable_updates", "hi_matvecs",
                                             "history_count", "rel_res", "ms"])}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "fem.h"', 'int main(void) {']
    for cs, (_, names) in fields.items():
        src.append(f'printf("%zu\\n", sizeof({cs}));')
        for nm in names:
            src.append(f'printf("%zu\\n", offsetof({cs}, {nm}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    k = 0
    for cs, (py, names) in fields.items():
        S = getattr(fem, py)
        assert ctypes.sizeof(S) == vals[k], cs
        k += 1
        for (pyname, _), nm in zip(S._fields_, names):
            assert getattr(S, pyname).offset == vals[k], (cs, nm)
            k += 1


def test_geo_layout_width(fem):
    # W: largest power of two dividing the points per direction, <= 16 bytes of values
    assert fem.fem_geo_vector_width(7, 0, fem.FEM_F64) == 2      # 8 GLL points, FP64
    assert fem.fem_geo_vector_width(7, 0, fem.FEM_F32) == 4
    assert fem.fem_geo_vector_width(7, 0, fem.FEM_BF16G64) == 8
    assert fem.fem_geo_vector_width(7, 1, fem.FEM_F64) == 1      # 9 GL points
    assert fem.fem_geo_vector_width(5, 1, fem.FEM_F16) == 1      # 7 GL points
    assert fem.fem_geo_vector_width(11, 0, fem.FEM_BF16) == 4    # 12 GLL points
    for n, W in ((8, 2), (8, 8), (12, 4), (9, 1)):
        off = fem.geo_layout_offsets(n, W)
        assert sorted(off) == list(range(n ** 3))                # a permutation
    off = fem.geo_layout_offsets(8, 2)
    assert off[0] == 0 and off[64] == 1 and off[1] == 2 and off[128] == 128


def test_tune_load(fem):
    before = fem.fem_tune_get(fem.FEM_OP_BP10, 7, fem.FEM_F64)
    fem.fem_tune_load("# op N prec epb cap\n0 7 0 3 0\n1 7 0 1 512  # comment\n\n")
    assert fem.fem_tune_get(fem.FEM_OP_BP10, 7, fem.FEM_F64) == (3, 0)
    assert fem.fem_tune_get(fem.FEM_OP_BP35, 7, fem.FEM_F64) == (1, 512)
    for bad, st in (("0 7 0 3\n", fem.FEM_ERR_ARG), ("0 7 0 999 0\n", fem.FEM_ERR_UNSUPPORTED),
                    ("0 16 0 1 0\n", fem.FEM_ERR_ARG), ("garbage\n", fem.FEM_ERR_ARG)):
        with pytest.raises(fem.FemError) as ei:
            fem.fem_tune_load("0 7 0 1 0\n" + bad)      # nothing applied on error
        assert ei.value.status == st
        assert fem.fem_tune_get(fem.FEM_OP_BP10, 7, fem.FEM_F64) == (3, 0)
    fem.fem_tune_load("0 7 0 0 0\n1 7 0 0 0\n")
    assert fem.fem_tune_get(fem.FEM_OP_BP10, 7, fem.FEM_F64)[0] == before[0]


def test_batch_validation_on_host(fem):
    d = fem.ApplyDesc(op=1, N=7, E=4, prec=0, D1d=0x1000, G=0x2000, u=0x3000, y=1 << 40)
    with pytest.raises(fem.FemError) as ei:
        fem.fem_batch_apply([d, fem.ApplyDesc(op=5, N=7, E=4)], stream=0)
    assert ei.value.status == fem.FEM_ERR_ARG
    with pytest.raises(fem.FemError):
        fem.BatchGraph([d], lanes=9, stream=0)


def test_build_id_matches_sources(fem):
    """The library reports the hash of the sources it was built from; a library
    that is stale against the checkout's csrc/ and include/ fails here."""
    from paper_1711_00903_amd import build
    assert fem.fem_build_id() == build.source_hash(), \
        "libfem.so was built from other sources: rebuild (__graft_entry__.build())"


def test_vertex_applies_reject_overlapping_fields(fem):
    """u and y of the vertex applies may not share bytes (partial overlap
    included): a workgroup would overwrite another element's input."""
    bad = 0x100000
    E, N = 4, 7
    nbytes = E * (N + 1) ** 3 * 8
    for shift in (16, nbytes - 16, -(nbytes - 16)):
        with pytest.raises(fem.FemError) as ei:
            fem.fem_stiff_collocated_vertex_apply(N, E, bad, bad, 0.0, bad + 2 * nbytes,
                                                  bad + 2 * nbytes + shift, stream=0)
        assert ei.value.status == fem.FEM_ERR_ARG, shift
        with pytest.raises(fem.FemError) as ei:
            fem.fem_stiff_dealiased_vertex_apply(N, E, bad, bad, bad, 0.0, bad + 2 * nbytes,
                                                 bad + 2 * nbytes + shift, stream=0)
        assert ei.value.status == fem.FEM_ERR_ARG, shift


def test_launch_size_limits(tmp_path):
    """Work-item count of one dispatch stays below 2^32: the grid clamp and
    the chunk loops of the element launchers (launch.hpp) cover every element
    exactly once for any element count up to the advertised limit."""
    import subprocess
    src = tmp_path / "grid.cpp"
    src.write_text(r'''
#include <cstdio>
#include "launch.hpp"
int main() {
    const int threads[] = {64, 128, 192, 256, 320, 384, 448, 512};
    const long long Es[] = {1, 7, 65535, 16777216, 67108865, 2147483647LL};
    for (int t : threads) {
        const long long g = fem::max_grid(t);
        if (g * t > 0xFFFFFFFFLL || (g + 1) * t <= 0xFFFFFFFFLL && g < 0x7FFFFFFFLL) { printf("bad %d\n", t); return 1; }
        for (long long E : Es) {
            // chunk loop of the line-per-lane launchers
            long long covered = 0, launches = 0;
            for (long long e0 = 0; e0 < E; e0 += g) {
                const long long grid = E - e0 < g ? E - e0 : g;
                if (grid * t > 0xFFFFFFFFLL || grid < 1) { printf("chunk %d %lld\n", t, E); return 1; }
                covered += grid; ++launches;
            }
            if (covered != E) { printf("cover %d %lld\n", t, E); return 1; }
        }
    }
    printf("ok\n");
    return 0;
}
''')
    exe = tmp_path / "grid"
    csrc = os.path.join(ROOT, "paper_1711_00903_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc,
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout


def test_assembly_inverse_map(fem):
    """The inverse of a gather map groups each global node's local copies in
    ascending order (a stable sort of the local indices by global node)."""
    import workloads
    gids, ng = workloads.global_numbering(3, 2, E=20)
    off, loc = fem.fem_assembly_inverse_map(gids, ng)
    order = np.argsort(gids.ravel(), kind="stable")
    np.testing.assert_array_equal(loc, order)
    np.testing.assert_array_equal(np.diff(off), np.bincount(gids.ravel(), minlength=ng))
    assert off[0] == 0 and off[-1] == gids.size
    bad = gids.copy()
    bad[3, 5] = ng
    with pytest.raises(fem.FemError) as ei:
        fem.fem_assembly_inverse_map(bad, ng)
    assert ei.value.status == fem.FEM_ERR_ARG


def test_assembled_validation(fem):
    bad = 0x1000
    op = fem.CgOperator(N=3, E=8, I1d=bad, D1d=bad, G=bad, wJ=bad, lam=1.0)
    asm = fem.Assembly(n_global=125, gather=bad, offsets=bad, locals=bad)
    assert fem.fem_assembled_workspace_bytes(op, asm) > 0
    asm.n_global = 8 * 64 + 1                                 # more global than local nodes
    assert fem.fem_assembled_workspace_bytes(op, asm) == 0
    asm.n_global = 125
    opt = fem.CgOptions(mode=1, rtol=1e-8, max_iters=10)
    with pytest.raises(fem.FemError) as ei:                  # FP64 only
        fem.fem_pcg_solve(op, asm, opt, None, bad, bad + 4096, bad, 1 << 30, stream=0)
    assert ei.value.status == fem.FEM_ERR_ARG
    opt.mode = 0
    with pytest.raises(fem.FemError) as ei:                  # workspace too small
        fem.fem_pcg_solve(op, asm, opt, None, bad, bad + 4096, 1 << 20, 256, stream=0)
    assert ei.value.status == fem.FEM_ERR_WORKSPACE
    with pytest.raises(fem.FemError) as ei:
        fem.fem_gather(64, 125, bad + 2, bad, 1 << 30, stream=0)
    assert ei.value.status == fem.FEM_ERR_ALIGN


def test_cg_noalloc_host_checks(fem):
    """fem_cg_solve_noalloc: the binding's array size is the header's, and a
    solve that needs more than the array, or a bad argument, is refused during
    validation (before any device work)."""
    txt = open(os.path.join(ROOT, "include", "fem.h")).read()
    m = re.search(r"#define FEM_CG_NOALLOC_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == fem.FEM_CG_NOALLOC_BYTES
    bad = 0x1000
    n7 = 512 * 8
    op = fem.CgOperator(N=7, E=4096, I1d=bad, D1d=bad, G=bad, wJ=bad, lam=1.0)
    opt = fem.CgOptions(mode=0, rtol=1e-8, max_iters=10)
    assert fem.fem_cg_workspace_bytes(op, opt) > fem.FEM_CG_NOALLOC_BYTES
    with pytest.raises(fem.FemError) as ei:
        fem.fem_cg_solve_noalloc(op, opt, bad, bad + 4096 * n7, stream=0)
    assert ei.value.status == fem.FEM_ERR_WORKSPACE
    op.E = 64
    assert fem.fem_cg_workspace_bytes(op, opt) <= fem.FEM_CG_NOALLOC_BYTES
    with pytest.raises(fem.FemError) as ei:                  # b and x overlap
        fem.fem_cg_solve_noalloc(op, opt, bad, bad + 16, stream=0)
    assert ei.value.status == fem.FEM_ERR_ARG
    opt.mode = 3
    with pytest.raises(fem.FemError) as ei:
        fem.fem_cg_solve_noalloc(op, opt, bad, bad + 64 * n7, stream=0)
    assert ei.value.status == fem.FEM_ERR_ARG

"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (plain C) is rebuilt with gcc and both sanitizers, preloaded into
  a fresh interpreter, and exercised through its Python wrappers: tables,
  geometry, node coordinates, the three operators with their lambda terms,
  the CG operator and its long-double residual, at N = 1, 3, 7 and 15.
* The library's host units (fem_api.cpp: argument validation, launch-shape
  model, tune table; basis.cpp: 1-D tables; batch.cpp: descriptor checks) are
  rebuilt with both sanitizers on their host side and linked with the other
  objects of the build; a sanitized C++ driver then makes every call that
  needs no GPU: the tables at N = 1..15, the launch-shape model for every
  (operator, N, precision, packing), applies rejected during validation, the
  assembled operator's inverse map with a bad entry, and the tune-table
  parser on a malformed line.
Device code is not sanitized: the GPU address sanitizer needs XNACK-enabled
code objects and runtime, which these MI355X machines run without.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libs(names):
    out = []
    for n in names:
        p = subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{n} not available")
        out.append(p)
    return out


ORACLE_EXERCISE = r"""
import sys, numpy as np
sys.path.insert(0, ROOT)
import oracle, workloads
oracle._LIB = LIB
oracle.lib.cache_clear()
oracle.set_threads(2)
for N in (1, 3, 7, 15):
    X = workloads.element_vertices(3, E=5)
    pb = oracle.Problem(N, X)
    u = np.random.default_rng(N).uniform(-1, 1, (5, (N + 1) ** 3))
    pb.mass(u); pb.stiff35(u, 0.5); pb.stiff30(u, 0.5); pb.cg_operator(u, 2.0)
    pb.cg_residual_ld(u, u, 1.0)
    oracle.node_coords(N, X, "gll"); oracle.node_coords(N, X, "gl")
assert oracle.lib()._name == LIB
print("ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                    "-o", lib, os.path.join(ROOT, "oracle", "fem_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=":".join(_libs(["libasan.so", "libubsan.so"])),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + ORACLE_EXERCISE
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


DRIVER = r"""
#include <dlfcn.h>
#include <cstdio>
#include <cstdint>
#include <vector>
#include "fem.h"
int main(int argc, char **argv) {
    void *h = dlopen(argv[1], RTLD_NOW);
    if (!h) { std::printf("dlopen: %s\n", dlerror()); return 1; }
    auto tables = (int (*)(int, double *, double *, double *, double *, double *, double *, double *))dlsym(h, "fem_basis_tables");
    auto inv = (int (*)(int64_t, const int32_t *, int64_t, int32_t *, int32_t *))dlsym(h, "fem_assembly_inverse_map");
    auto load = (int (*)(const char *))dlsym(h, "fem_tune_load");
    auto mass = (int (*)(int, int64_t, const double *, const void *, const void *, void *, double, int, float, void *))dlsym(h, "fem_mass_apply");
    auto kinfo = (int (*)(int, int, int, int, int *, int *))dlsym(h, "fem_kernel_info");
    auto sepb = (int (*)(int, int, int, int *, int))dlsym(h, "fem_supported_epb");
    if (!tables || !inv || !load || !mass || !kinfo || !sepb) { std::printf("missing symbol\n"); return 1; }
    for (int N = 1; N <= 15; ++N) {
        std::vector<double> a(N + 1), b(N + 1), c(N + 2), d(N + 2), I((N + 2) * (N + 1)), D((N + 1) * (N + 1)),
            Dg((N + 2) * (N + 2));
        if (tables(N, a.data(), b.data(), c.data(), d.data(), I.data(), D.data(), Dg.data())) return 2;
        for (int op = 0; op < 3; ++op)
            for (int p = 0; p < 9; ++p) {
                int e[4], th, lds;
                int n = sepb(op, N, p, e, 4);
                for (int q = 0; q < n && q < 4; ++q) kinfo(op, N, p, e[q], &th, &lds);
                kinfo(op, N, p, 0, &th, &lds);
            }
        if (mass(N, 8, (double *)0x1000, (void *)0x1000, (void *)0x2000, (void *)0x2008, 0.0, 0, 1.0f, nullptr) == 0) return 3;
    }
    std::vector<int32_t> g = {0, 1, 2, 1, 2, 3}, off(5), loc(6);
    if (inv(6, g.data(), 4, off.data(), loc.data())) return 4;
    g[3] = 7;
    if (inv(6, g.data(), 4, off.data(), loc.data()) == 0) return 5;
    load("0 7 0 1 0\n# comment\n1 7 0 4 0\nnot a line\n");
    std::printf("ok\n");
    return 0;
}
"""


@pytest.mark.slow
def test_library_host_units_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    build = os.path.join(ROOT, "_build")
    units = ["fem_api", "basis", "batch"]
    if not os.path.exists(hipcc) or not shutil.which("g++") or not os.path.isdir(build):
        pytest.skip("hipcc, g++ or the library build objects not available")
    others = sorted(os.path.join(build, f) for f in os.listdir(build)
                    if f.endswith(".o") and f[:-2] not in units)
    if len(others) < 30:
        pytest.skip("library build objects not available")
    objs = []
    for u in units:
        o = str(tmp_path / f"{u}.o")
        subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1711_00903_amd", "csrc"),
                        "-c", os.path.join(ROOT, "paper_1711_00903_amd", "csrc", u + ".cpp"), "-o", o],
                       check=True, capture_output=True)
        objs.append(o)
    lib = str(tmp_path / "libfem_san.so")
    subprocess.run(["g++", "-shared", "-fPIC", "-fsanitize=address,undefined", "-o", lib] + objs + others +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", exe, "-ldl"], check=True)
    r = subprocess.run([exe, lib], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]

"""CPU-only checks of the HIP library: it loads, exports every function its
header declares, validates arguments before touching the GPU, and its host
set-up (LGL basis and DSS line operators) is right.  No kernel runs here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1702_04316_amd import numa
from paper_1702_04316_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "numa.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\**\s*(numa_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = numa.load()
    names = _declared_functions()
    assert len(names) >= 14, names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps each of them under the same name (minus the prefix)
    for n in names:
        assert hasattr(numa, n[len("numa_"):]), n


def test_setup_rejects_bad_arguments_before_any_gpu_call():
    g, _ = numa.make_grid(1000.0, 1000.0, 1000.0, 2, 2, 2)
    bg = numa.numa_background(300.0, 1e5, 1004.67, 287.17, 9.80616)
    lib = numa.load()
    out = C.c_void_p()
    assert lib.numa_setup(None, 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    assert "NULL" in numa.last_error()
    assert lib.numa_setup(C.byref(g), 0, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    assert lib.numa_setup(C.byref(g), 9, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_UNSUPPORTED
    bad = numa.numa_grid(-1.0, 1000.0, 1000.0, 2, 2, 2, None)
    assert lib.numa_setup(C.byref(bad), 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    bad = numa.numa_grid(1000.0, 1000.0, 1000.0, 0, 2, 2, None)
    assert lib.numa_setup(C.byref(bad), 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    gz, keep = numa.make_grid(1000.0, 1000.0, 1000.0, 2, 2, 3, zface=[0.0, 500.0, 400.0, 1000.0])
    assert lib.numa_setup(C.byref(gz), 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    assert "increasing" in numa.last_error()
    tall, _ = numa.make_grid(1000.0, 1000.0, 40000.0, 2, 2, 2)
    assert lib.numa_setup(C.byref(tall), 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_ARG
    # 321 levels: the column solve of one 64-column workgroup would need more
    # than one CU's 160 KB of LDS
    long_col, _ = numa.make_grid(1000.0, 1000.0, 10000.0, 2, 2, 80)
    assert lib.numa_setup(C.byref(long_col), 4, C.byref(bg), None, C.byref(out)) == numa.NUMA_E_UNSUPPORTED
    assert "LDS" in numa.last_error()
    badbg = numa.numa_background(300.0, 1e5, 200.0, 287.17, 9.8)
    assert lib.numa_setup(C.byref(g), 4, C.byref(badbg), None, C.byref(out)) == numa.NUMA_E_ARG
    assert out.value is None
    # NULL-context calls
    assert lib.numa_destroy(None) == numa.NUMA_OK
    assert lib.numa_check(None) == numa.NUMA_E_ARG
    assert lib.numa_hevi_step(None, None, 1.0, 1) == numa.NUMA_E_ARG
    assert lib.numa_set_column_solver(None, numa.SOLVER_BLOCKED) == numa.NUMA_E_ARG
    assert lib.numa_imex3d_setup(None, 1.0, 30, 1, 30, 100) == numa.NUMA_E_ARG
    assert lib.numa_imex3d_step(None, None, 1.0, 1e-8, None) == numa.NUMA_E_ARG
    assert lib.numa_imex3d_solve(None, None, None, 1e-8, None) == numa.NUMA_E_ARG
    assert lib.numa_imex3d_bounds(None, None) == numa.NUMA_E_ARG
    assert lib.numa_imex3d_set_bounds(None, 1.0, 2.0) == numa.NUMA_E_ARG
    assert lib.numa_schur_apply(None, None, None) == numa.NUMA_E_ARG
    assert lib.numa_schur_rhs(None, None, None) == numa.NUMA_E_ARG
    assert lib.numa_pbno_apply(None, None, None) == numa.NUMA_E_ARG


@pytest.mark.parametrize("N", range(1, 16))
def test_library_lgl_basis(N):
    """The library's own LGL basis (Sturm bisection + barycentric D) against
    numpy's Legendre roots and polynomial exactness."""
    xi, D = numa.lgl_basis(N)
    inner = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real) if N > 1 else np.array([])
    ref = np.concatenate(([-1.0], inner, [1.0]))
    assert np.max(np.abs(xi - ref)) < 2e-15
    for k in range(0, N + 1):
        exact = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(D @ xi ** k - exact)) < 1e-12 * (N + 1) ** 2


def _apply_x(wxy, N, g_line):
    """Apply the periodic x line operator to one x-line of unique nodes."""
    nx = g_line.size
    out = np.zeros(nx)
    for i in range(nx):
        a = i % N
        start = i - a - N
        for m in range(2 * N + 1):
            out[i] += wxy[0, a, m] * g_line[(start + m) % nx]
    return out


@pytest.mark.parametrize("N,nex", [(3, 2), (4, 3), (5, 2), (8, 2)])
def test_line_operator_x_exact_on_c1_periodic_cubic(N, nex):
    lx = 3000.0
    g, _ = numa.make_grid(lx, 1000.0, 1000.0, nex, 1, 1)
    wxy, _ = numa.line_operators(g, N)
    grid = W.Grid(lx, 1000.0, 1000.0, nex, 1, 1, N)
    x, _, _ = W.node_coords(grid)
    f = x * (x - lx / 2) * (x - lx)
    df = 3 * x * x - 3 * lx * x + lx * lx / 2
    assert np.max(np.abs(_apply_x(wxy, N, f) - df)) < 1e-9 * np.max(np.abs(df))


@pytest.mark.parametrize("N,nez,seed", [(1, 4, 0), (2, 3, 1), (4, 10, 2), (7, 3, 3), (8, 2, 4)])
def test_line_operator_z_exact_on_polynomials(N, nez, seed):
    lz = 10000.0
    zf = W.random_zface(nez, lz, seed)
    g, keep = numa.make_grid(1000.0, 1000.0, lz, 1, 1, nez, zface=zf)
    _, dzb = numa.line_operators(g, N)
    grid = W.Grid(1000.0, 1000.0, lz, 1, 1, nez, N, zface=zf)
    _, _, z = W.node_coords(grid)
    nz = z.size
    s = z / lz
    for k in range(0, N + 1):
        p = s ** k
        dp = k * s ** (k - 1) / lz if k > 0 else np.zeros_like(s)
        out = np.zeros(nz)
        for r in range(nz):
            for m in range(2 * N + 1):
                kk = r - N + m
                if 0 <= kk < nz:
                    out[r] += dzb[r, m] * p[kk]
                else:
                    assert dzb[r, m] == 0.0
        assert np.max(np.abs(out - dp)) < 1e-10 / lz, (k, np.max(np.abs(out - dp)))


def test_line_operator_z_matches_oracle_dss(oracle_mod):
    """The library's column operator equals the oracle's element-local
    derivative + DSS (probed through the oracle's L_V with g = 0)."""
    lz = 6000.0
    N, nez = 4, 3
    zf = W.random_zface(nez, lz, 11)
    g, keep = numa.make_grid(1000.0, 1000.0, lz, 1, 1, nez, zface=zf)
    _, dzb = numa.line_operators(g, N)
    o = oracle_mod.Oracle(1000.0, 1000.0, lz, 1, 1, nez, N, grav=0.0, zface=zf)
    rho0 = o.background()["rho0"][0]
    nz = nez * N + 1
    Dz = np.zeros((nz, nz))
    for m in range(nz):
        q = np.zeros(o.shape)
        q[3, m] = 1.0
        Dz[:, m] = -o.lv(q)[0, :, 0, 0] / rho0
    band = np.zeros((nz, nz))
    for r in range(nz):
        for m in range(2 * N + 1):
            kk = r - N + m
            if 0 <= kk < nz:
                band[r, kk] = dzb[r, m]
    # w at the walls is zero in L_V's probe of w; compare the interior columns
    assert np.max(np.abs(band[:, 1:-1] - Dz[:, 1:-1])) < 1e-13 * np.max(np.abs(Dz))

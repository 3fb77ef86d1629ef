"""GPU tests of the precision form (numa_hevi_step_mixed): the first-stage
tendency R1 stored in FP32; FP64 state, accumulator, stage values,
right-hand-side arithmetic and column solves.

The bar is a relative L2 error per variable of at most 1e-6 against the
FP64 oracle after 100 steps, at N = 4 and N = 7, and against the FP64 step
(which equals the oracle to 1e-11) on the benchmarked grid after 100 steps.
The form's FP64 parts are checked exactly: a rest state stays at rest.
"""
import numpy as np
import pytest

from paper_1702_04316_amd import workloads as W

pytestmark = pytest.mark.gpu

BAR = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def numa_mod():
    from paper_1702_04316_amd import numa
    numa.load()
    return numa


def _rel(a, b):
    return np.array([np.linalg.norm(a[f] - b[f]) / np.linalg.norm(b[f]) for f in range(5)])


def _oracle(O, g, bg):
    return O.Oracle(g.lx, g.ly, g.lz, g.nex, g.ney, g.nez, g.N, theta0=bg.theta0, p00=bg.p00, cp=bg.cp,
                    rgas=bg.rgas, grav=bg.grav, zface=g.zface)


@pytest.mark.parametrize("name", ["box_small", "box_precision"])
def test_mixed_error_against_oracle(torch_cuda, numa_mod, oracle_mod, name):
    wl = W.box_small("R1") if name == "box_small" else W.box_precision("small")
    g = wl.grid
    q0 = W.make_initial_state(wl)
    o = _oracle(oracle_mod, g, wl.background)
    o.factor_dt(wl.dt)
    ref = o.step(q0, wl.dt, 100)
    ctx = numa_mod.Context(g, wl.background)
    ctx.factor(wl.dt)
    q = torch_cuda.from_numpy(q0.copy()).cuda()
    ctx.step(q, 100, mixed=True)
    ctx.check()
    e = _rel(q.cpu().numpy(), ref)
    print(f"{wl.name} mixed, 100 steps, rel L2 per variable (rho', u, v, w, theta'): {e}")
    assert np.all(e < BAR), e
    ctx.close()


def test_mixed_full_size_against_fp64(torch_cuda, numa_mod):
    """The benchmarked grid: 100 precision-form steps against 100 FP64 steps
    (the FP64 path equals the oracle to 1e-11)."""
    wl = W.box_large("R1")
    ctx = numa_mod.Context(wl.grid, wl.background)
    ctx.factor(wl.dt)
    q0 = torch_cuda.from_numpy(W.make_initial_state(wl)).cuda()
    a, b = q0.clone(), q0.clone()
    ctx.step(a, 100)
    ctx.step(b, 100, mixed=True)
    ctx.check()
    e = _rel(b.cpu().numpy(), a.cpu().numpy())
    print(f"box_large mixed vs FP64, 100 steps: {e}")
    assert np.all(e < BAR), e
    ctx.close()


def test_mixed_rest_state_stays_at_rest(torch_cuda, numa_mod):
    g = W.Grid(30000.0, 20000.0, 8000.0, 3, 2, 4, 4)
    ctx = numa_mod.Context(g)
    dt = W.dt_for_courant(g, 15.0, "z")
    ctx.factor(dt)
    q = torch_cuda.zeros(ctx.shape, dtype=torch_cuda.float64, device="cuda")
    ctx.step(q, 5, mixed=True)
    ctx.check()
    assert float(q.abs().max()) == 0.0
    ctx.close()


def test_mixed_error_codes(torch_cuda, numa_mod):
    g = W.Grid(30000.0, 20000.0, 8000.0, 3, 2, 4, 4)
    ctx = numa_mod.Context(g)
    q = torch_cuda.zeros(ctx.shape, dtype=torch_cuda.float64, device="cuda")
    lib = numa_mod.load()
    import ctypes as C
    assert lib.numa_hevi_step_mixed(ctx.ctx, C.c_void_p(q.data_ptr()), 1.0, 1) == numa_mod.NUMA_E_NOT_FACTORED
    ctx.factor(1.0)
    assert lib.numa_hevi_step_mixed(ctx.ctx, C.c_void_p(q.data_ptr()), 2.0, 1) == numa_mod.NUMA_E_DT_MISMATCH
    assert lib.numa_hevi_step_mixed(ctx.ctx, None, 1.0, 1) == numa_mod.NUMA_E_ARG
    ms = (C.c_double * 5)()
    assert lib.numa_profile_steps_mixed(ctx.ctx, C.c_void_p(q.data_ptr()), 1.0, 0, ms) == numa_mod.NUMA_E_ARG
    ctx.close()


# (N, nex, ney, nez, Nb): the blocked solve with four and eight wavefronts,
# the one-lane solve of a 161-level column, and a stratified background
# (whose solves also read R1's theta' as FP32)
SOLVE_GRIDS = [(3, 3, 2, 5, 0.0), (5, 2, 2, 13, 0.0), (4, 2, 2, 40, 0.0), (4, 3, 2, 6, 0.012)]


@pytest.mark.parametrize("N,nex,ney,nez,nbv", SOLVE_GRIDS)
def test_mixed_with_every_column_solver(torch_cuda, numa_mod, N, nex, ney, nez, nbv):
    """The precision form's solve shapes (R1 read as FP32) in every column
    solver: two steps within the 1e-6 bar of the FP64 step with the same
    solver, and the solvers' precision-form results equal to rounding."""
    lz = 6000.0 if nez <= 8 else 20000.0
    g = W.Grid(9000.0 * nex, 7000.0 * ney, lz, nex, ney, nez, N)
    bg = W.Background(nbv=nbv) if nbv else None
    dt = min(W.dt_for_courant(g, 15.0, "z"), W.dt_for_courant(g, 0.4, "x"), W.dt_for_courant(g, 0.4, "y"))
    q0 = W.make_random_state(g, 70 + N, wind=3.0)
    outs = {}
    for kind in (numa_mod.SOLVER_BAND, numa_mod.SOLVER_BLOCKED, numa_mod.SOLVER_PER_COLUMN):
        ctx = numa_mod.Context(g, bg)
        ctx.set_column_solver(kind)
        ctx.factor(dt)
        a = torch_cuda.from_numpy(q0.copy()).cuda()
        b = a.clone()
        ctx.step(a, 2)
        ctx.step(b, 2, mixed=True)
        ctx.check()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        e = _rel(b, a)
        print(f"N={N} nz={g.nz} Nb={nbv} solver {ctx.info()['column_solver']}: mixed vs FP64 {e}")
        assert np.all(e < BAR), (kind, e)
        outs[kind] = b
        ctx.close()
    for kind in (numa_mod.SOLVER_BLOCKED, numa_mod.SOLVER_PER_COLUMN):
        e = _rel(outs[kind], outs[numa_mod.SOLVER_BAND])
        assert np.all(e < 1e-12), (kind, e)


@pytest.mark.timeout(600)
def test_mixed_full_size_against_oracle(torch_cuda, numa_mod, oracle_mod):
    """The benchmarked grid (64x64x10 elements, N = 4, 2.7M unique nodes):
    the precision form against the oracle after each of 10 steps, every
    variable within the 1e-6 bar."""
    wl = W.box_large("R1")
    g = wl.grid
    q0 = W.make_initial_state(wl)
    o = _oracle(oracle_mod, g, wl.background)
    o.factor_dt(wl.dt)
    ctx = numa_mod.Context(g, wl.background)
    ctx.factor(wl.dt)
    q = torch_cuda.from_numpy(q0.copy()).cuda()
    qo = q0.copy()
    worst = np.zeros(5)
    for n in range(10):
        qo = o.step(qo, wl.dt, 1)
        ctx.step(q, 1, mixed=True)
        worst = np.maximum(worst, _rel(q.cpu().numpy(), qo))
    ctx.check()
    print(f"box_large mixed vs oracle, worst over 10 steps: {worst}")
    assert np.all(worst < BAR), worst
    ctx.close()
